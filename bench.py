#!/usr/bin/env python3
"""Throughput of the NMF-KL randomized coordinate-descent sweep on one MI355X.

One step = one outer iteration of Alg. 1 on the document-like corpus (50,000 words x
100,000 documents, ~13.2M nonzeros, r = 50): factor sums of W, the F-half over all
columns, factor sums of F, the W-half over all rows, and the float64 objective (eq. 1).
Inputs are resident in HBM before timing starts.  The metric is coordinate updates per
second, 2 * nnz * r per sweep (every nonzero takes part in r coordinate updates in each
half).

Prints one JSON line.  Besides the contract fields it carries:
  roofline      the dominant kernel's algorithmic (gather-model) bytes per launch over its
                average HIP-event duration, against the 8 TB/s HBM peak; traffic from the
                committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary when it was taken on the
                current kernel source, else null; valu_busy_pct likewise from the committed
                VALUBusy summary, and each group's valu_slots_per_update (64 x SQ_INSTS_VALU per
                coordinate update) from the committed instruction-count summary;
  cpu_baseline  the FP64 oracle timed on the host cores on a bounded sample (the first
                sweeps of the same workload from the same initial factors);
  sweep_ms      median, min and max of the timed sweeps (HIP events between steps);
  kernels       every timed launch group (ms per launch, GB/s under the gather model);
  check         the GPU objective after the first sweeps vs the oracle's on the same sweeps,
                and the factors after them (relative Frobenius error);
  batched       64 independent planted problems (n ~ U{1k..20k}, m ~ U{1k..50k}, r in
                {10, 16, 32, 64}, density 0.1-2%), 10 sweeps: one graph launch over the batch
                (mapping picked by the batch autotuner) against the 64 problems run one after
                another through plain handles;
  serving       fold-in requests (W 50,000 x 100 Gamma(0.1), Poisson arrivals at 20,000
                documents/s, log-normal lengths up to 5,000 words) through the continuously
                batched server, against per-request plain fold-in calls in arrival order:
                documents/s and p50/p99 latency from arrival to the host seeing the result.
"""
import argparse
import collections
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCE = os.path.join(ROOT, "paper_1604_04026_amd", "csrc", "nmfkl_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_NAMES = {"fused_F": "k_sweep_fused", "fused_W": "k_sweep_fused", "long_F": "k_sweep_long",
                "long_W": "k_sweep_long", "model": "k_model_objective", "terms": "k_model_terms",
                "sums_F": "k_permute_jobs", "sums_W": "k_permute_jobs"}


def source_hash() -> str:
    """Hash of the kernel source with comments and whitespace runs removed, so that counter
    summaries stay matched across comment edits and are dropped on any code change."""
    import re
    with open(KERNEL_SOURCE, encoding="utf-8") as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    text = " ".join(text.split())
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def traffic_for(group: str):
    """HBM bytes per launch from the committed counter summary, if it matches the source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    entry = t.get("groups", {}).get(group)
    if not entry or t.get("kernel_source_sha256_16") != source_hash():
        return None
    return entry.get("hbm_bytes_per_launch")


def valu_busy_for(group: str):
    """VALU-busy % of a launch group from the committed counter summary, if it matches the source."""
    try:
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "valu.json")) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != source_hash():
        return None
    return t.get("groups", {}).get(group)


def valu_slots_for(group: str):
    """VALU lane slots per coordinate update of a launch group from the committed
    SQ_INSTS_VALU summary, if it matches the source."""
    try:
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "insts.json")) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != source_hash():
        return None
    return t.get("groups", {}).get(group, {}).get("valu_lane_slots_per_update")


def cpu_baseline(prob, seconds: float, keep=(), min_sweeps: int = 0):
    """The oracle's sweeps for about `seconds` (and at least `min_sweeps`); also returns its
    objectives and its factors after each sweep count in `keep` (for the GPU check)."""
    import numpy as np
    import oracle
    W = prob.W0.astype(np.float64)
    F = prob.F0.astype(np.float64)
    D = []
    kept = {}
    t0 = time.perf_counter()
    sweeps = 0
    while True:
        ids = oracle.permutation(0, sweeps, 0, prob.r)
        F, _, _ = oracle.sweep_F(prob, W, F, ids)
        W, _, _ = oracle.sweep_W(prob, F, W, ids)
        D.append(oracle.objective(prob, W, F))
        sweeps += 1
        if sweeps in keep:
            kept[sweeps] = (W.copy(), F.copy())
        if (time.perf_counter() - t0 >= seconds and sweeps >= min_sweeps) or sweeps >= 60:
            break
    dt = time.perf_counter() - t0
    # the same oracle on one core: the F-half of the first sweep
    threads = oracle.threads()
    oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.sweep_F(prob, prob.W0.astype(np.float64), prob.F0.astype(np.float64), oracle.permutation(0, 0, 0, prob.r))
    d1 = time.perf_counter() - t1
    oracle.set_threads(threads)
    return {"value": 2.0 * prob.nnz * prob.r * sweeps / dt, "unit": "updates/s",
            "cores": threads, "kind": "oracle",
            "sample": f"{sweeps} full sweeps (F-half + W-half + objective) of the same corpus from "
                      f"the same initial factors, {dt:.1f} s wall",
            "single_core": {"value": prob.nnz * prob.r / d1, "unit": "updates/s", "cores": 1,
                            "sample": f"the first F-half on one thread, {d1:.1f} s wall"}}, D, kept


def sweep_leg(P, prob, args, log):
    import torch
    dev = P.upload(prob, "cuda:0")
    h = P.nmfkl_create(dev, P.nmfkl_params_default(seed=args.seed, collect_timings=1, tuning=args.tuning))
    torch.cuda.synchronize()
    log("[bench] handle created")
    D_warm = []
    for t in range(args.warmup):
        P.nmfkl_sweep_F(h, t)
        P.nmfkl_sweep_W(h, t)
        D_warm.append(P.nmfkl_objective_carried(h))
    P.nmfkl_reset_timings(h)
    warm_factors = (dev.W.cpu().numpy(), dev.F.cpu().numpy())
    log(f"[bench] warmup done, D = {D_warm}")
    torch.cuda.synchronize()
    # one event per step on the handle's (default) stream: per-sweep times
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t_start = time.perf_counter()
    evs[0].record()
    # each step: both halves and eq. 1 on the device; the objective's value is copied to pinned
    # host memory on the stream and read once at the end (no host round trip per step)
    for i, t in enumerate(range(args.warmup, args.warmup + args.steps)):
        P.nmfkl_sweep_F(h, t)
        P.nmfkl_sweep_W(h, t)
        P.nmfkl_objective_enqueue(h)
        evs[i + 1].record()
    D = P.nmfkl_objective_read(h)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    sweep_ms = [evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)]
    tim = P.nmfkl_get_timings(h)
    final = (D, P.nmfkl_objective(h), dev.W.cpu().numpy(), dev.F.cpu().numpy())
    P.nmfkl_destroy(h)
    del dev
    log(f"[bench] timed {args.steps} sweeps in {elapsed * 1e3:.2f} ms, final D = {D}")
    return elapsed, tim, D_warm, sweep_ms, warm_factors, final


def batched_leg(P, probs, log):
    """10 sweeps of every problem: batch graph vs 64 sequential plain handles."""
    import numpy as np
    import torch
    sweeps = 10
    nnz = sum(p.nnz for p in probs)
    updates = 2.0 * sweeps * sum(p.nnz * p.r for p in probs)
    # plain: each problem's sweeps through its own handle, one problem after another
    devs = [P.upload(p, "cuda:0") for p in probs]
    hs = [P.nmfkl_create(d, P.nmfkl_params_default()) for d in devs]
    for h in hs:                       # warm-up sweeps (model values, caches)
        for t in range(sweeps):
            P.nmfkl_sweep_F(h, t)
            P.nmfkl_sweep_W(h, t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for h in hs:
        for t in range(sweeps, 2 * sweeps):
            P.nmfkl_sweep_F(h, t)
            P.nmfkl_sweep_W(h, t)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    D_plain = np.array([P.nmfkl_objective_carried(h) for h in hs])
    for h in hs:
        P.nmfkl_destroy(h)
    del hs, devs
    torch.cuda.empty_cache()
    log(f"[bench] batched: plain sequential {t_plain * 1e3:.1f} ms")
    # batch: autotune the mapping, warm-up run (captures the graph), timed run
    devs = [P.upload(p, "cuda:0") for p in probs]
    b = P.nmfkl_batch_create(devs)
    t0 = time.perf_counter()
    chosen = P.nmfkl_batch_tune(b, 0)
    t_tune = time.perf_counter() - t0
    P.nmfkl_batch_run(b, 0, sweeps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.nmfkl_batch_run(b, sweeps, sweeps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    D_batch = P.nmfkl_batch_objective(b)
    info = P.nmfkl_batch_get_info(b)
    P.nmfkl_batch_destroy(b)
    del devs
    torch.cuda.empty_cache()
    log(f"[bench] batched: graph {t_batch * 1e3:.1f} ms (tuner {t_tune:.2f} s, {info})")
    rel = np.abs(D_batch - D_plain) / D_plain
    return {
        "workload": "64 planted problems: n ~ U{1k..20k}, m ~ U{1k..50k}, r in {10,16,32,64}, "
                    "density U[0.1%,2%], Gamma(0.1) factors, 10 sweeps",
        "nprob": len(probs), "nnz_total": int(nnz), "sweeps": sweeps,
        "batch_ms": round(t_batch * 1e3, 3), "plain_sequential_ms": round(t_plain * 1e3, 3),
        "speedup": round(t_plain / t_batch, 3),
        "batch_updates_per_s": updates / t_batch, "plain_updates_per_s": updates / t_plain,
        "tuned": {"bin_shift": int(chosen.bin_shift), "tuning": int(chosen.tuning), "tuner_s": round(t_tune, 3)},
        "graph_cooperative": info["graph_cooperative"],
        "objective_rel_diff_batch_vs_plain_max": float(f"{rel.max():.2e}"),
        "timed": "sweeps 10..19 of every problem after 10 warm-up sweeps (graph captured in the warm-up)",
    }


def serving_leg(P, W, arrivals, ptr, idx, val, window_s, log):
    """Open-loop Poisson arrivals through the server, then per-request plain fold-in."""
    import numpy as np
    import torch
    Wd = torch.from_numpy(W).cuda()
    m = P.nmfkl_model_create(Wd)
    N = len(arrivals)
    r = W.shape[1]

    def doc(d):
        return idx[ptr[d]:ptr[d + 1]], val[ptr[d]:ptr[d + 1]]

    # ---- server: continuous batching
    srv = P.nmfkl_server_create(m, 512 << 20, lanes=8, lane_docs=256)
    buf = P.PollBuffer(4096, r)
    lat = np.full(N, np.nan)
    passes = np.zeros(N, np.int32)
    deferred = np.zeros(N, bool)     # refused at least once because the memory budget was full
    waiting = collections.deque()
    nxt, ndone, rejected = 0, 0, 0
    t0 = time.monotonic() + 0.05
    deadline = t0 + arrivals[-1] + 120.0
    while ndone + rejected < N:
        now = time.monotonic()
        while nxt < N and t0 + arrivals[nxt] <= now:
            waiting.append(nxt)
            nxt += 1
        while waiting:
            d = waiting[0]
            try:
                if P.nmfkl_server_submit(srv, d, *doc(d)) != 0:    # memory budget or waiting slots full
                    deferred[d] = True
                    break
            except P.NmfklError:
                rejected += 1        # refused for good (malformed or beyond the fold-in limits)
            waiting.popleft()
        k = P.nmfkl_server_poll_into(srv, buf)
        for q in range(k):
            rec = buf.res[q]
            lat[rec.req_id] = rec.t_done - (t0 + arrivals[rec.req_id])
            passes[rec.req_id] = rec.passes
        ndone += k
        if now > deadline:
            raise RuntimeError("serving leg did not drain")
    t_end = time.monotonic()
    P.nmfkl_server_destroy(srv)
    served_s = t_end - t0
    srv_out = {"docs": N, "wall_s": round(served_s, 3), "docs_per_s": ndone / served_s,
               "p50_ms": float(np.nanpercentile(lat, 50) * 1e3), "p99_ms": float(np.nanpercentile(lat, 99) * 1e3),
               "p999_ms": float(np.nanpercentile(lat, 99.9) * 1e3),
               "passes_median": float(np.median(passes)), "passes_max": int(passes.max()),
               "rejected": int(rejected), "deferred_by_admission": int(deferred.sum())}
    log(f"[bench] serving: server {srv_out}")

    # ---- plain: one nmfkl_foldin call per request, in arrival order, for window_s seconds
    lat_p = []
    t0 = time.monotonic() + 0.05
    d = 0
    while d < N:
        now = time.monotonic()
        if now - t0 > window_s:
            break
        if t0 + arrivals[d] > now:
            continue
        i, v = doc(d)
        dp = torch.tensor([0, len(i)], dtype=torch.int64, device="cuda")
        di = torch.from_numpy(i).cuda()
        dv = torch.from_numpy(v).cuda()
        F, ps, kl = P.nmfkl_foldin(m, dp, di, dv)
        _ = F.cpu()
        lat_p.append(time.monotonic() - (t0 + arrivals[d]))
        d += 1
    t_p = time.monotonic() - t0
    lat_p = np.array(lat_p)
    plain_out = {"docs_completed": int(d), "window_s": round(t_p, 3), "docs_per_s": d / t_p,
                 "p50_ms": float(np.percentile(lat_p, 50) * 1e3), "p99_ms": float(np.percentile(lat_p, 99) * 1e3),
                 "arrived_in_window": int(np.searchsorted(arrivals, t_p))}
    log(f"[bench] serving: plain {plain_out}")
    P.nmfkl_model_destroy(m)
    return {
        "workload": f"fold-in: W 50000x{r} Gamma(0.1) resident; {N} Poisson requests at {N / arrivals[-1]:.0f}/s, "
                    "lengths LogNormal(ln 80, 1) in [1, 5000], Zipf(1.1) words, 1+Geometric(0.6) counts; "
                    "relative KL tolerance 1e-5",
        "server": srv_out, "plain_per_request": plain_out,
        "throughput_ratio": round(srv_out["docs_per_s"] / plain_out["docs_per_s"], 2),
        "latency": "arrival time to the host observing the finished document (H2D/D2H included)",
    }


COPY_BYTES = 256 << 20   # calibration copy of the traffic run


def traffic_run(args):
    """The command profiled for HBM traffic: a plain 256 MiB device copy (three times), then
    warm-up and timed sweeps of the corpus.  Run under rocprofv3 --pmc FETCH_SIZE, then
    under --pmc WRITE_SIZE; --traffic-summarize turns the two outputs into traffic.json."""
    from paper_1604_04026_amd import workloads
    prob = workloads.config(1, seed=args.seed)
    import torch
    import paper_1604_04026_amd as P
    torch.cuda.set_device(0)
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    dev = P.upload(prob, "cuda:0")
    h = P.nmfkl_create(dev, P.nmfkl_params_default(seed=args.seed, collect_timings=1))
    for t in range(1 + args.steps):
        P.nmfkl_sweep_F(h, t)
        P.nmfkl_sweep_W(h, t)
        P.nmfkl_objective_carried(h)
    tim = P.nmfkl_get_timings(h)
    P.nmfkl_destroy(h)
    print(json.dumps({"sweeps": 1 + args.steps, "gather_bytes": {k: v["gather_bytes"] for k, v in tim.items()},
                      "updates": {k: v["updates"] for k, v in tim.items()}}), flush=True)


def _counter_rows(path):
    import csv
    import glob
    files = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {path}")
    with open(files[0]) as fh:
        return list(csv.DictReader(fh))


GROUP_NAMES = ("fused_F", "fused_W", "long_F", "long_W", "terms")


def launch_groups(rows):
    """Per-dispatch values (dispatch id, kernel name, grid, value) of a --traffic-run ->
    per-launch-group values of the sweeps after the warm-up sweep.  In each half the
    long-segment launches are enqueued before the binned launch, and the binned launches
    alternate F-half, W-half; so a half's long-segment dispatches are those since the previous
    binned dispatch, and the objective's terms follow the W-half.  A group's value per sweep is
    the sum over its dispatches."""
    sweeps, pending_long, nfused = [], 0.0, 0
    for _, name, _, v in sorted(rows):
        if "k_sweep_long" in name:
            pending_long += v
        elif "k_sweep_fused" in name:
            half = "F" if nfused % 2 == 0 else "W"
            if half == "F":
                sweeps.append({g: 0.0 for g in GROUP_NAMES})
            sweeps[-1]["fused_" + half] += v
            sweeps[-1]["long_" + half] += pending_long
            pending_long = 0.0
            nfused += 1
        elif "k_model_terms" in name and sweeps:
            sweeps[-1]["terms"] += v
    sweeps = sweeps[1:]      # the warm-up sweep (first model pass, first touches)
    return {g: [sw[g] for sw in sweeps if sw[g] > 0] for g in GROUP_NAMES}


def valu_summarize(valu_dir, out_path):
    """VALUBusy and VALUUtilization (rocprofv3 derived counters, %) of each launch group of a
    --traffic-run, averaged over the sweeps after the warm-up sweep (a group of several
    dispatches: weighted by dispatch duration)."""
    rows = [r for r in _counter_rows(valu_dir)]
    per = collections.defaultdict(dict)
    meta = {}
    for r in rows:
        d = int(r["Dispatch_Id"])
        per[d][r["Counter_Name"]] = float(r["Counter_Value"])
        meta[d] = (r["Kernel_Name"], int(r.get("End_Timestamp", 0) or 0) - int(r.get("Start_Timestamp", 0) or 0))
    out_groups = {}
    for counter in ("VALUBusy", "VALUUtilization"):
        vals = [(d, meta[d][0], meta[d][1], per[d].get(counter, 0.0) * max(meta[d][1], 1)) for d in sorted(per)]
        durs = [(d, meta[d][0], meta[d][1], float(max(meta[d][1], 1))) for d in sorted(per)]
        num, den = launch_groups(vals), launch_groups(durs)
        for g in GROUP_NAMES:
            if num[g] and den[g]:
                out_groups.setdefault(g, {})[counter] = round(sum(num[g]) / sum(den[g]), 1)
    out = {"kernel_source_sha256_16": source_hash(),
           "counter": "rocprofv3 derived VALUBusy (100 * SQ_ACTIVE_INST_VALU / CU_NUM / GRBM_GUI_ACTIVE) and "
                      "VALUUtilization, per launch group, duration-weighted over the sweeps after the warm-up sweep of "
                      "bench.py --traffic-run --steps 3",
           "groups": {g: v["VALUBusy"] for g, v in out_groups.items() if "VALUBusy" in v},
           "utilization": {g: v.get("VALUUtilization") for g, v in out_groups.items()},
           "command": "rocprofv3 --pmc VALUBusy VALUUtilization -d <dir> -o run --output-format csv -- "
                      "python3 bench.py --traffic-run --steps 3; python3 bench.py --valu-summarize <dir> profiles/valu.json"}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def insts_summarize(insts_dir, run_log, out_path):
    """SQ_INSTS_VALU and SQ_INSTS_SALU (wave instructions) of each launch group of a
    --traffic-run, per launch (mean over the sweeps after the warm-up sweep), and VALU lane
    slots per coordinate update: 64 x VALU wave instructions / (nonzeros x r).  run_log is the
    traffic run's output, whose JSON line holds each group's updates per launch."""
    rows = _counter_rows(insts_dir)
    with open(run_log) as fh:
        info = json.loads([ln for ln in fh.read().splitlines() if ln.startswith("{")][-1])
    updates = info["updates"]
    groups = {}
    for counter in ("SQ_INSTS_VALU", "SQ_INSTS_SALU"):
        vals = [(int(r["Dispatch_Id"]), r["Kernel_Name"], 0, float(r["Counter_Value"]))
                for r in rows if r.get("Counter_Name") == counter]
        for g, v in launch_groups(vals).items():
            if v:
                groups.setdefault(g, {})[counter.lower() + "_per_launch"] = sum(v) / len(v)
    for g, d in groups.items():
        u = updates.get(g) or 0.0
        if u > 0 and "sq_insts_valu_per_launch" in d:
            d["valu_lane_slots_per_update"] = round(64.0 * d["sq_insts_valu_per_launch"] / u, 2)
        d["updates_per_launch"] = u
    out = {"kernel_source_sha256_16": source_hash(),
           "counter": "SQ_INSTS_VALU and SQ_INSTS_SALU (wave instructions) per launch group of bench.py --traffic-run "
                      "--steps 3, mean over the sweeps after the warm-up sweep; lane slots per update = 64 x VALU "
                      "instructions / (nonzeros x r)",
           "groups": groups,
           "command": "rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU -d <dir> -o run --output-format csv -- python3 "
                      "bench.py --traffic-run --steps 3 > <log>; python3 bench.py --insts-summarize <dir> <log> "
                      "profiles/insts.json"}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def traffic_summarize(fetch_dir, write_dir, out_path):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the traffic run -> bytes per launch of
    each launch group, scaled by what the counters read for the calibration copy."""
    def per_dispatch(rows, counter):
        out = []
        for r in rows:
            if r.get("Counter_Name") != counter:
                continue
            out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], int(r.get("Grid_Size", 0) or 0),
                        float(r["Counter_Value"])))
        out.sort()
        return out
    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = per_dispatch(_counter_rows(d), counter)
        copies = [v for _, name, _, v in rows if "copy" in name.lower() or "elementwise" in name.lower()]
        copies = [v for v in copies if v > 0.25 * COPY_BYTES / 1024]
        if not copies:
            raise SystemExit(f"{counter}: calibration copy not found")
        scale = (COPY_BYTES / 1024) / (sum(copies[1:] or copies) / len(copies[1:] or copies))
        groups = launch_groups(rows)
        res[counter] = {"scale": scale, "copy_kib": copies,
                        "groups": {g: (sum(v) / len(v) * 1024 * scale if v else None) for g, v in groups.items()}}
    groups = {}
    for g in GROUP_NAMES:
        f, w = res["FETCH_SIZE"]["groups"][g], res["WRITE_SIZE"]["groups"][g]
        groups[g] = {"fetch_bytes_per_launch": f, "write_bytes_per_launch": w,
                     "hbm_bytes_per_launch": (f + w) if f is not None and w is not None else None}
    out = {"kernel_source_sha256_16": source_hash(),
           "calibration": {"copy_bytes": COPY_BYTES, "fetch_scale": res["FETCH_SIZE"]["scale"],
                           "write_scale": res["WRITE_SIZE"]["scale"]},
           "groups": groups,
           "commands": ["rocprofv3 --pmc FETCH_SIZE -d <fetch_dir> -o run --output-format csv -- "
                        "python3 bench.py --traffic-run --steps 3",
                        "rocprofv3 --pmc WRITE_SIZE -d <write_dir> -o run --output-format csv -- "
                        "python3 bench.py --traffic-run --steps 3",
                        "python3 bench.py --traffic-summarize <fetch_dir> <write_dir> profiles/traffic.json"]}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def large_problem(args, log):
    from paper_1604_04026_amd import workloads
    t0 = time.perf_counter()
    prob = workloads.config(2, seed=args.seed, workers=args.workers,
                            progress=lambda msg: log(f"[large] {msg} ({time.perf_counter() - t0:.0f} s)"))
    log(f"[large] generated n={prob.n} m={prob.m} r={prob.r} nnz={prob.nnz} ({time.perf_counter() - t0:.1f} s)")
    return prob


def large_leg(P, prob, args, log, sweeps: int = 10):
    """The large corpus (100,000 x 2,000,000, r = 100, ~300M nonzeros): `sweeps` outer
    iterations with float32 tiles and with bfloat16-stored tiles from the same initial factors
    (time per iteration, gather-model fraction of HBM peak per launch group and per iteration,
    the exact objective of each and their difference), and the first iteration's float32
    F-half and W-half checked on sampled columns and rows (the 20 heaviest rows included)
    against the oracle."""
    import numpy as np
    import torch
    from concurrent.futures import ThreadPoolExecutor
    res = {}
    first = None
    for bf in (0, 1):
        dev = P.upload(prob, "cuda:0")
        h = P.nmfkl_create(dev, P.nmfkl_params_default(seed=args.seed, tile_bf16=bf, collect_timings=1))
        P.nmfkl_sweep_F(h, 0)
        if bf == 0:
            Fg = dev.F.cpu().numpy()
        P.nmfkl_sweep_W(h, 0)
        if bf == 0:
            first = (Fg, dev.W.cpu().numpy())
        D1 = P.nmfkl_objective(h)
        P.nmfkl_reset_timings(h)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for t in range(1, sweeps):
            P.nmfkl_sweep_F(h, t)
            P.nmfkl_sweep_W(h, t)
        torch.cuda.synchronize()
        el = time.perf_counter() - ts
        tim = P.nmfkl_get_timings(h)
        D = P.nmfkl_objective(h)
        P.nmfkl_destroy(h)
        del dev
        torch.cuda.empty_cache()
        ms = el * 1e3 / (sweeps - 1)
        groups = {k: {"ms": round(v["ms_total"] / v["launches"], 4),
                      "frac": round(v["gather_bytes"] / (v["ms_total"] / v["launches"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
                  for k, v in tim.items() if v["launches"]}
        step_bytes = sum(v["gather_bytes"] * v["launches"] for v in tim.values()) / (sweeps - 1)
        res[bf] = {"ms_per_sweep": round(ms, 3), "updates_per_s": 2.0 * prob.nnz * prob.r / (ms * 1e-3),
                   "step_frac": round(step_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "objective_after_first_sweep": D1, "objective": D, "sweeps": sweeps, "groups": groups}
        log(f"[large] tile_bf16={bf}: {res[bf]}")
    # sampled parity of the first sweep (float32 tiles) against the oracle, columns and rows in
    # parallel threads (each oracle call releases the GIL)
    import oracle
    Fg, Wg = first
    ids = oracle.permutation(args.seed, 0, 0, prob.r)
    W0, F0 = prob.W0.astype(np.float64), prob.F0.astype(np.float64)
    rng = np.random.default_rng(7)
    sumW = oracle.factor_sums(W0)
    cols = np.sort(rng.choice(prob.m, 500, replace=False))
    F1 = Fg.astype(np.float64)
    sumF = oracle.factor_sums(F1)
    R = np.diff(prob.csr_ptr)
    heavy = np.sort(np.argsort(R)[-20:])
    rows = np.unique(np.concatenate([heavy, rng.choice(prob.n, 100, replace=False)]))
    with ThreadPoolExecutor(max_workers=16) as ex:
        Fo = np.array(list(ex.map(lambda j: oracle.alg2(prob.csc_idx[prob.csc_ptr[j]:prob.csc_ptr[j + 1]],
                                                        prob.csc_val[prob.csc_ptr[j]:prob.csc_ptr[j + 1]], W0, sumW,
                                                        F0[j], ids)[0], cols)))
        Wo = np.array(list(ex.map(lambda i: oracle.alg2(prob.csr_idx[prob.csr_ptr[i]:prob.csr_ptr[i + 1]],
                                                        prob.csr_val[prob.csr_ptr[i]:prob.csr_ptr[i + 1]], F1, sumF,
                                                        W0[i], ids)[0], rows)))

    def rowmax(g, o):
        e = np.linalg.norm(g.astype(np.float64) - o, axis=1) / np.maximum(np.linalg.norm(o, axis=1), 1e-300)
        return float(f"{e.max():.2e}")

    rel = lambda a, b: float(f"{np.linalg.norm(a.astype(np.float64) - b) / np.linalg.norm(b):.2e}")
    return {"workload": "large corpus 100000x2000000 r=100 (lognormal lengths median 92, cap 2000, Zipf(1.1) words, "
                        "1+Geometric(0.6) counts)",
            "n": prob.n, "m": prob.m, "r": prob.r, "nnz": prob.nnz, "longest_row": int(R.max()),
            "timed": f"iterations 2..{sweeps} (sums + both halves, no objective) after the first",
            "float32_tiles": res[0], "bf16_tiles": res[1],
            "bf16_objective_rel_diff": float(f"{abs(res[1]['objective'] - res[0]['objective']) / res[0]['objective']:.2e}"),
            "sampled_parity_first_sweep": {"F_rel": rel(Fg[cols], Fo), "F_col_rel_max": rowmax(Fg[cols], Fo),
                                           "cols": int(cols.size),
                                           "W_rel": rel(Wg[rows], Wo), "W_row_rel_max": rowmax(Wg[rows], Wo),
                                           "rows": int(rows.size),
                                           "heaviest_rows": [int(R[i]) for i in heavy]}}


def large_run(args, log):
    """bench.py --large: the large-corpus leg alone."""
    prob = large_problem(args, log)
    import torch
    import paper_1604_04026_amd as P
    torch.cuda.set_device(0)
    print(json.dumps(large_leg(P, prob, args, log)), flush=True)


def ablation_run(args, log):
    """The inner-loop readings and the L1 weight on the corpus, 10 outer iterations each from
    the same initial factors: objective (eq. 1) and the fraction of exact zeros in W and F.
    Settings: the build's reading (|step| break test, descent guard); the signed break test as
    printed; no guard; both as printed; and L1 weights beta_W = beta_F in {10, 100, 1000}."""
    from paper_1604_04026_amd import workloads
    prob = workloads.config(1, seed=args.seed)
    import numpy as np
    import torch
    import paper_1604_04026_amd as P
    torch.cuda.set_device(0)
    settings = [("reading (|step| break, guard)", {}), ("signed break as printed", {"literal_break": 1}),
                ("no descent guard", {"guard": 0}), ("signed break, no guard", {"literal_break": 1, "guard": 0})]
    settings += [(f"L1 beta_W = beta_F = {b:g}", {"beta_W": b, "beta_F": b}) for b in (10.0, 100.0, 1000.0)]
    out = {"workload": "doc-like corpus 50000x100000 r=50", "sweeps": 10, "runs": []}
    for name, kw in settings:
        dev = P.upload(prob, "cuda:0")
        h = P.nmfkl_create(dev, P.nmfkl_params_default(seed=args.seed, collect_stats=1, **kw))
        D = []
        for t in range(10):
            P.nmfkl_sweep_F(h, t)
            P.nmfkl_sweep_W(h, t)
            D.append(P.nmfkl_objective(h))
        st = P.nmfkl_get_stats(h)
        W, F = dev.W.cpu().numpy(), dev.F.cpu().numpy()
        P.nmfkl_destroy(h)
        rec = {"setting": name, "params": kw, "objective": D, "zeros_W": st["zeros_W"] / W.size,
               "zeros_F": st["zeros_F"] / F.size, "monotone": all(D[i + 1] <= D[i] for i in range(9)),
               "stats": st}
        log(f"[ablation] {name}: D10 {D[-1]:.6g} zeros W {rec['zeros_W']:.3f} F {rec['zeros_F']:.3f}")
        out["runs"].append(rec)
    print(json.dumps(out), flush=True)


def out_of_core_run(args, log):
    """The corpus with V in pinned host memory, streamed per half-sweep through two device
    staging buffers in chunks of 2M nonzeros (7 chunks per half): time per outer iteration
    against the in-HBM handle, PCIe bytes per iteration, and the objective of both."""
    from paper_1604_04026_amd import workloads
    prob = workloads.config(1, seed=args.seed)
    import torch
    import paper_1604_04026_amd as P
    torch.cuda.set_device(0)
    res = {}
    for ooc in (0, 1):
        dev = P.upload_host_v(prob) if ooc else P.upload(prob, "cuda:0")
        prm = P.nmfkl_params_default(seed=args.seed, out_of_core=ooc, ooc_chunk_nnz=1 << 21)
        h = P.nmfkl_create(dev, prm)
        for t in range(args.warmup):
            P.nmfkl_sweep_F(h, t)
            P.nmfkl_sweep_W(h, t)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for t in range(args.warmup, args.warmup + args.steps):
            P.nmfkl_sweep_F(h, t)
            P.nmfkl_sweep_W(h, t)
        torch.cuda.synchronize()
        el = time.perf_counter() - ts
        D = P.nmfkl_objective(h)
        P.nmfkl_destroy(h)
        del dev
        res[ooc] = {"ms_per_sweep": el * 1e3 / args.steps,
                    "updates_per_s": 2.0 * prob.nnz * prob.r * args.steps / el, "objective": D}
        log(f"[ooc] out_of_core={ooc}: {res[ooc]}")
    v_bytes = 2 * (prob.nnz * 8) + (prob.n + prob.m + 2) * 8
    out = {"workload": "doc-like corpus 50000x100000 r=50, V streamed from pinned host memory in chunks of "
                       "2097152 nonzeros", "sweeps_timed": args.steps,
           "in_hbm": res[0], "out_of_core": res[1],
           "h2d_bytes_per_sweep": v_bytes,
           "h2d_GBps_effective": v_bytes / (res[1]["ms_per_sweep"] * 1e-3) / 1e9,
           "objective_rel_diff": abs(res[1]["objective"] - res[0]["objective"]) / res[0]["objective"]}
    print(json.dumps(out), flush=True)


def main():
    if len(sys.argv) >= 2 and sys.argv[1] == "--traffic-summarize":
        traffic_summarize(sys.argv[2], sys.argv[3], sys.argv[4])
        return
    if len(sys.argv) >= 2 and sys.argv[1] == "--valu-summarize":
        valu_summarize(sys.argv[2], sys.argv[3])
        return
    if len(sys.argv) >= 2 and sys.argv[1] == "--insts-summarize":
        insts_summarize(sys.argv[2], sys.argv[3], sys.argv[4])
        return
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=100_000)
    ap.add_argument("--serving-rate", type=float, default=20_000.0, help="offered fold-in requests per second")
    ap.add_argument("--plain-window", type=float, default=3.0, help="seconds of per-request plain fold-in")
    ap.add_argument("--workers", type=int, default=16, help="processes generating the batched problems")
    ap.add_argument("--tuning", type=int, default=0, help="nmfkl_params.tuning bits (result-neutral)")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--traffic-run", action="store_true",
                    help="the command profiled for HBM traffic (calibration copy + sweeps only)")
    ap.add_argument("--no-large", action="store_true", help="skip the large-corpus leg of the default run")
    ap.add_argument("--large", action="store_true",
                    help="the large corpus (100,000 x 2,000,000, r = 100): float32 vs bf16 tiles")
    ap.add_argument("--out-of-core", action="store_true",
                    help="the corpus with V streamed from pinned host memory vs in HBM")
    ap.add_argument("--ablation", action="store_true",
                    help="inner-loop readings and L1 weights on the corpus: objective and exact zeros")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sweep's sharding over "
              "several GPUs is described as a design only and is not implemented.", file=sys.stderr)
        sys.exit(2)
    if args.traffic_run:
        traffic_run(args)
        return
    if args.out_of_core:
        out_of_core_run(args, (lambda *a: None) if args.quiet else (lambda *a: print(*a, file=sys.stderr, flush=True)))
        return
    if args.ablation:
        ablation_run(args, (lambda *a: None) if args.quiet else (lambda *a: print(*a, file=sys.stderr, flush=True)))
        return
    if args.large:
        large_run(args, (lambda *a: None) if args.quiet else (lambda *a: print(*a, file=sys.stderr, flush=True)))
        return

    from paper_1604_04026_amd import workloads

    log = (lambda *a: None) if args.quiet else (lambda *a: print(*a, file=sys.stderr, flush=True))
    # every workload is generated before the process touches the GPU (the batched members in
    # forked workers)
    t0 = time.perf_counter()
    prob = workloads.config(1, seed=args.seed)
    log(f"[bench] corpus generated: n={prob.n} m={prob.m} r={prob.r} nnz={prob.nnz} "
        f"({time.perf_counter() - t0:.1f} s)")
    batched = None
    if not args.no_batched:
        t0 = time.perf_counter()
        batched = workloads.batched_configs(seed=args.seed, workers=args.workers)
        log(f"[bench] 64 batched problems generated, nnz {sum(p.nnz for p in batched)} "
            f"({time.perf_counter() - t0:.1f} s)")
    serving = None
    if not args.no_serving:
        t0 = time.perf_counter()
        W = workloads.serving_model(seed=args.seed)
        arrivals, sptr, sidx, sval = workloads.serving_requests(args.serving_requests, rate=args.serving_rate,
                                                                 seed=args.seed)
        serving = (W, arrivals, sptr, sidx, sval)
        log(f"[bench] {args.serving_requests} serving requests generated ({time.perf_counter() - t0:.1f} s)")

    large = None if args.no_large else large_problem(args, log)

    import torch
    import paper_1604_04026_amd as P
    torch.cuda.set_device(0)

    elapsed, tim, D_warm, sweep_ms, warm_factors, final = sweep_leg(P, prob, args, log)
    updates = 2.0 * prob.nnz * prob.r * args.steps
    kernels = {}
    for name, k in tim.items():
        if k["launches"] == 0:
            continue
        ms = k["ms_total"] / k["launches"]
        kernels[name] = {"kernel": KERNEL_NAMES[name], "ms_per_launch": round(ms, 5),
                         "launches": int(k["launches"]), "gather_bytes": k["gather_bytes"],
                         "gather_GBps": round(k["gather_bytes"] / (ms * 1e-3) / 1e9, 1) if ms > 0 else None}
    # Roofline under the gather model.  The dominant kernel is the one with the most algorithmic
    # bytes per step over all its launch groups (the long-segment groups included); its achieved
    # rate is its algorithmic bytes per launch over its average launch duration.  Every launch
    # group's fraction and the whole step's (all bytes of a step over ms_per_step) are reported
    # beside it.
    per_kernel = collections.defaultdict(lambda: {"bytes": 0.0, "ms": 0.0, "launches": 0, "groups": []})
    for g, k in kernels.items():
        pk = per_kernel[k["kernel"]]
        pk["bytes"] += k["gather_bytes"] * k["launches"]
        pk["ms"] += k["ms_per_launch"] * k["launches"]
        pk["launches"] += k["launches"]
        pk["groups"].append(g)
    dname = max(per_kernel, key=lambda n: per_kernel[n]["bytes"])
    dk = per_kernel[dname]
    achieved = dk["bytes"] / (dk["ms"] * 1e-3) / 1e9
    tr = [traffic_for(g) for g in dk["groups"]]
    traffic = (sum(tr) / len(tr)) if all(x is not None for x in tr) else None
    vb = [valu_busy_for(g) for g in dk["groups"]]
    valu = (round(sum(v * kernels[g]["ms_per_launch"] for v, g in zip(vb, dk["groups"])) /
                  sum(kernels[g]["ms_per_launch"] for g in dk["groups"]), 1)
            if all(v is not None for v in vb) else None)
    step_bytes = sum(k["gather_bytes"] * k["launches"] for k in kernels.values()) / args.steps
    step_ms = elapsed * 1e3 / args.steps
    roofline = {"bound": "hbm", "kernel": f"{dname} ({' + '.join(dk['groups'])})", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "valu_busy_pct": valu,
                "bytes_model": "gather model: per nonzero 8 + 4r, per segment 8 + 8r",
                "step": {"gather_bytes": step_bytes, "ms": round(step_ms, 4),
                         "achieved_GBps": round(step_bytes / (step_ms * 1e-3) / 1e9, 1),
                         "frac": round(step_bytes / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
                "groups": {g: {"frac": round(k["gather_GBps"] / HBM_PEAK_GBS, 4), "ms": k["ms_per_launch"],
                               "valu_busy_pct": valu_busy_for(g), "valu_slots_per_update": valu_slots_for(g)}
                           for g, k in kernels.items()}}

    out = {
        "metric": "nnz·r CD updates/sec per sweep",
        "value": updates / elapsed,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "doc-like corpus 50000x100000 r=50 (lognormal lengths median 80, "
                               "Zipf(1.1) words, 1+Geometric(0.6) counts)",
                   "n": prob.n, "m": prob.m, "r": prob.r, "nnz": prob.nnz, "seed": args.seed,
                   "tuning": args.tuning,
                   "step": "sumW + F-half + sumF + W-half + float64 objective (eq. 1 from the "
                           "carried float64 model values)"},
        "roofline": roofline,
        "sweep_ms": {"median": round(statistics.median(sweep_ms), 4), "min": round(min(sweep_ms), 4),
                     "max": round(max(sweep_ms), 4), "source": "HIP events between steps on the handle's stream"},
        "kernels": kernels,
    }
    if batched is not None:
        out["batched"] = batched_leg(P, batched, log)
    if serving is not None:
        W, arrivals, sptr, sidx, sval = serving
        out["serving"] = serving_leg(P, W, arrivals, sptr, sidx, sval, args.plain_window, log)
    if not args.no_cpu_baseline:
        import numpy as np
        n_all = args.warmup + args.steps
        base, D_orc, kept = cpu_baseline(prob, args.cpu_seconds, keep=(args.warmup, n_all), min_sweeps=n_all)
        out["cpu_baseline"] = base
        n_cmp = min(len(D_orc), len(D_warm))
        rel = [abs(D_warm[i] - D_orc[i]) / D_orc[i] for i in range(n_cmp)]
        check = {"sweeps_compared": n_cmp, "objective_rel_err_vs_oracle": [float(f"{x:.2e}") for x in rel]}

        def factor_errors(gpu, orc):
            fe = {}
            for name, g, o in (("W", gpu[0], orc[0]), ("F", gpu[1], orc[1])):
                g = g.astype(np.float64)
                rows = np.linalg.norm(g - o, axis=1) / np.maximum(np.linalg.norm(o, axis=1), 1e-300)
                flip = np.any((g == 0) != (o == 0), axis=1)
                fe[name] = {"rel_frobenius": float(f"{np.linalg.norm(g - o) / np.linalg.norm(o):.2e}"),
                            "row_rel_max_no_flip": float(f"{rows[~flip].max():.2e}") if (~flip).any() else 0.0,
                            "rows_over_1e-4": int(np.sum(rows > 1e-4)), "rows_with_zero_flip": int(flip.sum())}
            return fe

        if args.warmup in kept and n_cmp == len(D_warm):
            check["factor_rel_err_vs_oracle"] = factor_errors(warm_factors, kept[args.warmup])
        if n_all in kept and len(D_orc) >= n_all:
            D_end, D_exact, Wg, Fg = final
            check["after_all_sweeps"] = {
                "sweeps": n_all,
                "objective_rel_err_vs_oracle": float(f"{abs(D_end - D_orc[n_all - 1]) / D_orc[n_all - 1]:.2e}"),
                "exact_objective_rel_err_vs_oracle": float(f"{abs(D_exact - D_orc[n_all - 1]) / D_orc[n_all - 1]:.2e}"),
                "factors": factor_errors((Wg, Fg), kept[n_all])}
        out["check"] = check
    if large is not None:
        out["large"] = large_leg(P, large, args, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
