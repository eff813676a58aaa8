"""Host-side helpers of bench.py: the HBM-traffic summary from rocprofv3 counter files."""
import csv
import json
import os

import pytest

import bench

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _write(path, counter, copy_kib, fused_kib, terms_kib, long_kib=(30.0, 20.0, 50.0)):
    os.makedirs(path, exist_ok=True)
    rows, d = [], 0

    def add(name, v):
        nonlocal d
        d += 1
        rows.append({**{f: 0 for f in FIELDS}, "Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter,
                     "Counter_Value": v})
    for _ in range(3):
        add("__amd_rocclr_copyBuffer", copy_kib)
    for sweep in range(4):               # each half: sums, long-segment launches, binned launch; then the terms
        add("nmfkl::k_permute_jobs(...)", 7.0)
        add("void nmfkl::k_sweep_long_flat<20, 256, 2>(...)", long_kib[0])
        add("void nmfkl::k_sweep_fused<false>(...)", fused_kib[0])
        add("nmfkl::k_permute_jobs(...)", 7.0)
        add("void nmfkl::k_sweep_long_flat<20, 256, 2>(...)", long_kib[1])
        add("nmfkl::k_zero_u64(...)", 1.0)
        add("void nmfkl::k_sweep_long_queue<20, 512, 1>(...)", long_kib[2])
        add("void nmfkl::k_sweep_fused<false>(...)", fused_kib[1])
        add("nmfkl::k_permute_jobs(...)", 7.0)
        add("nmfkl::k_model_terms(...)", terms_kib)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        w.writerows(rows)


def test_traffic_summary_scales_by_the_copy(tmp_path):
    half = bench.COPY_BYTES / 1024 / 2          # a counter that sees half the bytes
    _write(tmp_path / "f", "FETCH_SIZE", half, (1000.0, 500.0), 100.0)
    _write(tmp_path / "w", "WRITE_SIZE", 2 * half, (80.0, 40.0), 1.0)
    out = tmp_path / "traffic.json"
    bench.traffic_summarize(str(tmp_path / "f"), str(tmp_path / "w"), str(out))
    t = json.loads(out.read_text())
    assert t["calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert t["calibration"]["write_scale"] == pytest.approx(1.0)
    g = t["groups"]
    assert g["fused_F"]["fetch_bytes_per_launch"] == pytest.approx(2000.0 * 1024)
    assert g["fused_W"]["fetch_bytes_per_launch"] == pytest.approx(1000.0 * 1024)
    assert g["fused_F"]["hbm_bytes_per_launch"] == pytest.approx((2000.0 + 80.0) * 1024)
    assert g["terms"]["fetch_bytes_per_launch"] == pytest.approx(200.0 * 1024)
    assert g["long_F"]["fetch_bytes_per_launch"] == pytest.approx(60.0 * 1024)
    assert g["long_W"]["fetch_bytes_per_launch"] == pytest.approx(140.0 * 1024)
    assert t["kernel_source_sha256_16"] == bench.source_hash()


def test_valu_summary_weights_dispatches_by_duration(tmp_path):
    path = tmp_path / "v"
    os.makedirs(path)
    rows, d = [], 0

    def add(name, busy, util, dur):
        nonlocal d
        d += 1
        for counter, v in (("VALUBusy", busy), ("VALUUtilization", util)):
            rows.append({**{f: 0 for f in FIELDS}, "Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter,
                         "Counter_Value": v, "Start_Timestamp": 1000 * d, "End_Timestamp": 1000 * d + dur})
    for sweep in range(3):
        add("void nmfkl::k_sweep_long_flat<20, 256, 2>(...)", 40.0, 90.0, 100)
        add("void nmfkl::k_sweep_fused<false>(...)", 70.0, 85.0, 1000)
        add("void nmfkl::k_sweep_long_flat<20, 256, 2>(...)", 50.0, 90.0, 100)
        add("void nmfkl::k_sweep_long_queue<20, 512, 1>(...)", 30.0, 90.0, 300)
        add("void nmfkl::k_sweep_fused<false>(...)", 80.0, 80.0, 500)
        add("nmfkl::k_model_terms(...)", 60.0, 99.0, 50)
    with open(path / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        w.writerows(rows)
    out = tmp_path / "valu.json"
    bench.valu_summarize(str(path), str(out))
    v = json.loads(out.read_text())
    assert v["groups"]["fused_F"] == pytest.approx(70.0)
    assert v["groups"]["long_W"] == pytest.approx((50.0 * 100 + 30.0 * 300) / 400, abs=0.05)
    assert v["utilization"]["fused_W"] == pytest.approx(80.0)
    assert v["kernel_source_sha256_16"] == bench.source_hash()


def test_insts_summary_per_update(tmp_path):
    """VALU wave instructions per launch group (mean over the sweeps after the warm-up
    sweep; a half's long launches add up) and lane slots per update = 64 x instructions over
    the group's nonzeros x r, which come from the traffic run's JSON line."""
    path = tmp_path / "i"
    os.makedirs(path)
    rows, d = [], 0

    def add(name, valu, salu):
        nonlocal d
        d += 1
        for counter, v in (("SQ_INSTS_VALU", valu), ("SQ_INSTS_SALU", salu)):
            rows.append({**{f: 0 for f in FIELDS}, "Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter,
                         "Counter_Value": v})
    for sweep in range(4):
        scale = 9.0 if sweep == 0 else 1.0   # the warm-up sweep is left out
        add("void nmfkl::k_sweep_fused<false>(...)", 1000.0 * scale, 10.0)
        add("void nmfkl::k_sweep_long_flat<20, 256, 2>(...)", 300.0, 5.0)
        add("void nmfkl::k_sweep_long_queue<20, 512, 1>(...)", 100.0, 5.0)
        add("void nmfkl::k_sweep_fused<false>(...)", 500.0, 10.0)
        add("nmfkl::k_model_terms(...)", 50.0, 1.0)
    with open(path / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        w.writerows(rows)
    log = tmp_path / "run.log"
    log.write_text("[bench] noise\n" + json.dumps({"sweeps": 4, "updates": {"fused_F": 640.0, "fused_W": 320.0,
                                                                          "long_W": 1280.0, "terms": 0.0}}) + "\n")
    out = tmp_path / "insts.json"
    bench.insts_summarize(str(path), str(log), str(out))
    g = json.loads(out.read_text())["groups"]
    assert g["fused_F"]["sq_insts_valu_per_launch"] == pytest.approx(1000.0)
    assert g["fused_F"]["valu_lane_slots_per_update"] == pytest.approx(100.0)
    assert g["fused_W"]["valu_lane_slots_per_update"] == pytest.approx(100.0)
    assert g["long_W"]["sq_insts_valu_per_launch"] == pytest.approx(400.0)
    assert g["long_W"]["valu_lane_slots_per_update"] == pytest.approx(20.0)
    assert "valu_lane_slots_per_update" not in g["terms"]
