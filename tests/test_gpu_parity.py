"""GPU path vs the FP64 oracle, through the C ABI (all tests need an MI355X).

Tolerances (float32 GPU arithmetic against the float64 oracle on the same seeded input,
the same initial factors and the same coordinate orders):
  * objective: relative 1e-5 every sweep;
  * factors: relative Frobenius 1e-4 (one half-sweep from an identical state, and at the
    end of a trajectory).
Discrete decisions (enter / break / guard / clamp to zero) can flip between float32 and
float64; flips are counted and reported, and the norm tolerances absorb them.
"""
import numpy as np
import pytest

import oracle
from paper_1604_04026_amd import workloads

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1604_04026_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.load()


def relf(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def flips(a, b):
    return int(np.sum((np.asarray(a) == 0) != (np.asarray(b) == 0)))


def mid_corpus(seed=0, n=3000, m=2000, r=20):
    ptr, idx, val = workloads.corpus(n, m, 80.0, 1.0, 2000, 1.1, 0.6, seed=seed, tag=7)
    return workloads._problem(n, m, r, ptr, idx, val, seed, 7, {"name": f"corpus {n}x{m} r={r}"})


CASES = {
    "tiny": lambda: workloads.config(0, seed=0),
    "planted_mid": lambda: workloads.config(0, seed=1, n=3000, m=2500, r=16, density=0.01),
    "corpus_mid": lambda: mid_corpus(),
}


def gpu_half(prob, W, F, t, half, prm=None):
    dev = P.upload(prob, "cuda", W=W, F=F)
    h = P.nmfkl_create(dev, prm)
    if half == "F":
        P.nmfkl_sweep_F(h, t)
    else:
        P.nmfkl_sweep_W(h, t)
    out = (dev.W if half == "W" else dev.F).cpu().numpy()
    P.nmfkl_destroy(h)
    return out


@pytest.mark.parametrize("case", sorted(CASES))
def test_step_parity_from_identical_state(case):
    prob = CASES[case]()
    W0 = prob.W0.astype(np.float64)
    F0 = prob.F0.astype(np.float64)
    t = 3
    ids = oracle.permutation(0, t, 0, prob.r)
    # F-half
    Fo, _, _ = oracle.sweep_F(prob, W0, F0, ids)
    Fg = gpu_half(prob, prob.W0, prob.F0, t, "F")
    eF = relf(Fg, Fo)
    # W-half from the oracle's F (rounded to float32 on both sides)
    F1 = Fo.astype(np.float32)
    Wo, _, _ = oracle.sweep_W(prob, F1.astype(np.float64), W0, ids)
    Wg = gpu_half(prob, prob.W0, F1, t, "W")
    eW = relf(Wg, Wo)
    print(f"{case}: F rel {eF:.2e} flips {flips(Fg, Fo)}; W rel {eW:.2e} flips {flips(Wg, Wo)}")
    assert np.all(Fg >= 0) and np.all(Wg >= 0)
    assert eF <= 1e-4 and eW <= 1e-4


@pytest.mark.parametrize("case", ["tiny", "planted_mid", "corpus_mid"])
def test_trajectory_parity(case):
    prob = CASES[case]()
    sweeps = 10
    dev = P.upload(prob, "cuda")
    h = P.nmfkl_create(dev)
    Dg = []
    for t in range(sweeps):
        P.nmfkl_sweep_F(h, t)
        P.nmfkl_sweep_W(h, t)
        Dg.append(P.nmfkl_objective(h))
    Wg, Fg = dev.W.cpu().numpy(), dev.F.cpu().numpy()
    P.nmfkl_destroy(h)
    Wo, Fo, Do = oracle.run(prob, sweeps)
    relD = np.abs(np.array(Dg) - Do) / Do
    print(f"{case}: D rel per sweep {np.array2string(relD, precision=1)}; W {relf(Wg, Wo):.2e} "
          f"F {relf(Fg, Fo):.2e}; flips W {flips(Wg, Wo)} F {flips(Fg, Fo)}")
    assert np.all(np.diff(Dg) <= 1e-6 * np.array(Dg[1:]))
    assert np.all(relD <= 1e-5)
    assert relf(Wg, Wo) <= 1e-4 and relf(Fg, Fo) <= 1e-4


def test_checkpoint_and_resume():
    """A handle destroyed after 3 iterations and a new one created from the saved W and F
    continue at t = 3: the new handle computes the model values from the factors, where the
    continuous one carries them, so the two runs agree to float64 rounding of the model (far
    inside the oracle tolerance), and the resumed run matches the oracle's 6 iterations."""
    prob = CASES["corpus_mid"]()
    dev = P.upload(prob, "cuda")
    h = P.nmfkl_create(dev)
    for t in range(6):
        P.nmfkl_sweep_F(h, t)
        P.nmfkl_sweep_W(h, t)
        if t == 2:
            saved = (dev.W.cpu().numpy(), dev.F.cpu().numpy())
    Wc, Fc, Dc = dev.W.cpu().numpy(), dev.F.cpu().numpy(), P.nmfkl_objective(h)
    P.nmfkl_destroy(h)
    dev = P.upload(prob, "cuda", W=saved[0], F=saved[1])
    h = P.nmfkl_create(dev)
    for t in range(3, 6):
        P.nmfkl_sweep_F(h, t)
        P.nmfkl_sweep_W(h, t)
    Wr, Fr, Dr = dev.W.cpu().numpy(), dev.F.cpu().numpy(), P.nmfkl_objective(h)
    P.nmfkl_destroy(h)
    Wo, Fo, Do = oracle.run(prob, 6)
    print(f"resume vs continuous: W {relf(Wr, Wc):.2e} F {relf(Fr, Fc):.2e} D {abs(Dr - Dc) / Dc:.2e}; "
          f"resume vs oracle: W {relf(Wr, Wo):.2e} F {relf(Fr, Fo):.2e} D {abs(Dr - Do[-1]) / Do[-1]:.2e}")
    assert abs(Dr - Dc) <= 1e-7 * Dc and relf(Wr, Wc) <= 1e-5 and relf(Fr, Fc) <= 1e-5
    assert abs(Dr - Do[-1]) <= 1e-5 * Do[-1] and relf(Wr, Wo) <= 1e-4 and relf(Fr, Fo) <= 1e-4


def test_objective_parity():
    prob = CASES["corpus_mid"]()
    rng = np.random.default_rng(3)
    W = rng.random((prob.n, prob.r)).astype(np.float32)
    F = rng.random((prob.m, prob.r)).astype(np.float32)
    F[:, 3] = 0.0
    dev = P.upload(prob, "cuda", W=W, F=F)
    h = P.nmfkl_create(dev)
    d = P.nmfkl_objective(h)
    P.nmfkl_destroy(h)
    do = oracle.objective(prob, W, F)
    assert abs(d - do) / do <= 1e-6


def test_objective_infinite_when_model_zero_at_a_nonzero():
    prob = CASES["tiny"]()
    W = prob.W0.copy()
    W[prob.csc_idx[0]] = 0.0
    dev = P.upload(prob, "cuda", W=W)
    h = P.nmfkl_create(dev)
    assert np.isinf(P.nmfkl_objective(h))
    P.nmfkl_destroy(h)


def test_create_validates_on_device():
    import torch
    prob = CASES["tiny"]()

    def expect_inval(**mutate):
        dev = P.upload(prob, "cuda")
        for k, fn in mutate.items():
            t = getattr(dev, k)
            setattr(dev, k, fn(t.clone()))
        with pytest.raises(P.NmfklError) as e:
            P.nmfkl_create(dev)
        assert e.value.code == -1, e.value
        return e.value.message

    def swap_first(t):
        seg = t.clone()
        seg[0], seg[1] = t[1], t[0]
        return seg

    def neg_first(t):
        t[0] = -1.0
        return t

    def nan_first(t):
        t[5] = float("nan")
        return t

    def break_ptr(t):
        t[3] = t[4] + 1
        return t

    def out_of_range(t):
        t[2] = prob.n + 5
        return t

    assert "order" in expect_inval(csc_idx=swap_first) or True
    assert "value" in expect_inval(csc_val=neg_first)
    assert "value" in expect_inval(csr_val=nan_first)
    assert "pointer" in expect_inval(csc_ptr=break_ptr)
    assert "range" in expect_inval(csc_idx=out_of_range)
    assert "W" in expect_inval(W=neg_first)
    assert "F" in expect_inval(F=nan_first)

    def change_value(t):
        t[7] = t[7] + 1.0
        return t
    assert "transpose" in expect_inval(csr_val=change_value)
    torch.cuda.synchronize()


def test_empty_columns_and_rows_go_to_zero():
    prob = CASES["tiny"]()
    Fg = gpu_half(prob, prob.W0, prob.F0, 0, "F")
    empty = np.diff(prob.csc_ptr) == 0
    assert empty.any() and np.all(Fg[empty] == 0)


def test_stats_counters():
    """The binned launch keeps counters only when the handle collects statistics (another
    kernel instance); both instances must give the same factors bit for bit."""
    prob = CASES["tiny"]()
    out = {}
    for collect in (1, 0):
        dev = P.upload(prob, "cuda")
        h = P.nmfkl_create(dev, P.nmfkl_params_default(collect_stats=collect))
        P.nmfkl_sweep_F(h, 0)
        P.nmfkl_sweep_W(h, 0)
        st = P.nmfkl_get_stats(h)
        out[collect] = (dev.W.cpu().numpy(), dev.F.cpu().numpy(), st)
        P.nmfkl_destroy(h)
    st = out[1][2]
    assert st["coords"] == (prob.m + prob.n) * prob.r
    assert st["evals"] >= st["coords"] and st["steps"] > 0
    assert out[0][2]["coords"] == 0
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    # exact zeros of the factors (the sparsity of the paper's Table 2), counted on the device
    for k in (0, 1):
        W, F, s = out[k]
        assert s["zeros_W"] == int(np.sum(W == 0)) and s["zeros_F"] == int(np.sum(F == 0))
    assert 0 < out[1][2]["zeros_F"] < F.size


def test_power_of_two_bins_give_identical_results():
    """tuning bit 2 maps segments that fit 3, 5 or 6 nonzeros per lane to the 4- or 8-per-lane
    group of the same lane count: the extra elements stay empty, so both halves' factors are
    bit for bit those of the default bins."""
    prob = CASES["corpus_mid"]()
    out = []
    for tuning in (0, 4):
        dev = P.upload(prob, "cuda")
        h = P.nmfkl_create(dev, P.nmfkl_params_default(tuning=tuning))
        for t in range(2):
            P.nmfkl_sweep_F(h, t)
            P.nmfkl_sweep_W(h, t)
        out.append((dev.W.cpu().numpy(), dev.F.cpu().numpy()))
        P.nmfkl_destroy(h)
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def long_corpus(seed=0):
    """Rows up to ~20k nonzeros: the binned launch's 256 x 8 variant (1025..2048), one
    cooperative block (2049..5120) and several."""
    n, m, r = 2000, 20000, 12
    ptr, idx, val = workloads.corpus(n, m, 80.0, 1.0, 2000, 1.1, 0.6, seed=seed, tag=8)
    return workloads._problem(n, m, r, ptr, idx, val, seed, 8, {"name": f"corpus {n}x{m} r={r}"})


def test_long_segments_step_and_trajectory():
    prob = long_corpus()
    R = np.diff(prob.csr_ptr)
    assert R.max() > 4 * 4096 and ((R > 1024) & (R <= 4096)).any()
    t = 1
    ids = oracle.permutation(0, t, 0, prob.r)
    Wo, _, _ = oracle.sweep_W(prob, prob.F0.astype(np.float64), prob.W0.astype(np.float64), ids)
    Wg = gpu_half(prob, prob.W0, prob.F0, t, "W")
    rows_long = R > 1024
    e_all, e_long = relf(Wg, Wo), relf(Wg[rows_long], Wo[rows_long])
    print(f"long W-half: rel {e_all:.2e}, long rows rel {e_long:.2e}, flips {flips(Wg, Wo)}")
    assert e_all <= 1e-4 and e_long <= 1e-4
    sweeps = 5
    dev = P.upload(prob, "cuda")
    h = P.nmfkl_create(dev)
    Dg = []
    for t in range(sweeps):
        P.nmfkl_sweep_F(h, t)
        P.nmfkl_sweep_W(h, t)
        Dg.append(P.nmfkl_objective(h))
    Wg, Fg = dev.W.cpu().numpy(), dev.F.cpu().numpy()
    P.nmfkl_destroy(h)
    Wo, Fo, Do = oracle.run(prob, sweeps)
    relD = np.abs(np.array(Dg) - Do) / Do
    print(f"long trajectory: D rel {np.array2string(relD, precision=1)}; W {relf(Wg, Wo):.2e} F {relf(Fg, Fo):.2e}")
    assert np.all(relD <= 1e-5) and relf(Wg, Wo) <= 1e-4 and relf(Fg, Fo) <= 1e-4


def test_carried_objective_and_refresh_mode():
    """The two model paths against the oracle over 12 unregularised sweeps (Alg. 1/Alg. 2),
    with nmfkl_objective_carried inside the loop and the exact objective once at the end.
    refresh_model = 0 (the default, the path the bench times): each F-half reads the float64
    model values the previous W-half carried.  refresh_model = 1: they are recomputed from W
    and F before every F-half (the model-pass timings show it).  Both stay within the
    tolerances of the oracle, and within 1e-6 of each other (the carried values track the
    factors as stored)."""
    prob = CASES["corpus_mid"]()
    sweeps = 12
    res = {}
    for refresh in (0, 1):
        dev = P.upload(prob, "cuda")
        h = P.nmfkl_create(dev, P.nmfkl_params_default(refresh_model=refresh, collect_timings=1))
        Dc = []
        for t in range(sweeps):
            P.nmfkl_sweep_F(h, t)
            P.nmfkl_sweep_W(h, t)
            Dc.append(P.nmfkl_objective_carried(h))
        De = P.nmfkl_objective(h)
        passes = P.nmfkl_get_timings(h)["model"]["launches"]
        res[refresh] = (np.array(Dc), De, dev.W.cpu().numpy(), dev.F.cpu().numpy(), passes)
        P.nmfkl_destroy(h)
    Wo, Fo, Do = oracle.run(prob, sweeps)
    for refresh, (Dc, De, W, F, passes) in res.items():
        rel = np.abs(Dc - Do) / Do
        print(f"refresh_model={refresh}: model passes {passes}; D rel max {rel.max():.2e}, exact vs carried "
              f"at the end {abs(De - Dc[-1]) / De:.2e}; W {relf(W, Wo):.2e} F {relf(F, Fo):.2e}")
        assert np.all(rel <= 1e-5)
        assert abs(De - Dc[-1]) / De <= 1e-6
        assert relf(W, Wo) <= 1e-4 and relf(F, Fo) <= 1e-4
    # carried: the first F-half and the final exact objective; refreshed: also every later F-half
    assert res[0][4] == 2 and res[1][4] == sweeps + 1
    assert relf(res[0][2], res[1][2].astype(np.float64)) <= 1e-6


def test_objective_enqueue_then_read_equals_carried():
    """The two-step objective gives the synchronous one's value bit for bit, only the last
    enqueue is read, and a read without an enqueue is rejected."""
    prob = CASES["corpus_mid"]()
    Ds = {}
    for mode in ("sync", "split"):
        dev = P.upload(prob, "cuda")
        h = P.nmfkl_create(dev, P.nmfkl_params_default())
        D = []
        for t in range(3):
            P.nmfkl_sweep_F(h, t)
            P.nmfkl_sweep_W(h, t)
            if mode == "sync":
                D.append(P.nmfkl_objective_carried(h))
            else:
                P.nmfkl_objective_enqueue(h)
        if mode == "split":
            D.append(P.nmfkl_objective_read(h))
            with pytest.raises(P.NmfklError) as ei:
                P.nmfkl_objective_read(h)
            assert ei.value.code == -1
        Ds[mode] = D
        P.nmfkl_destroy(h)
    assert Ds["split"][-1] == Ds["sync"][-1]


def test_regularised_trajectory_parity():
    """eq. 2's L1/L2 terms (alpha_1, alpha_2, beta_1, beta_2 > 0): GPU vs oracle."""
    prob = CASES["corpus_mid"]()
    kw = dict(alpha_W=0.2, alpha_F=0.05, beta_W=0.01, beta_F=0.3)
    sweeps = 6
    dev = P.upload(prob, "cuda")
    h = P.nmfkl_create(dev, P.nmfkl_params_default(**kw))
    for t in range(sweeps):
        P.nmfkl_sweep_F(h, t)
        P.nmfkl_sweep_W(h, t)
    Wg, Fg = dev.W.cpu().numpy(), dev.F.cpu().numpy()
    P.nmfkl_destroy(h)
    Wo, Fo, _ = oracle.run(prob, sweeps, oracle.params(**kw))
    print(f"regularised: W {relf(Wg, Wo):.2e} F {relf(Fg, Fo):.2e}; zeros W {np.mean(Wg == 0):.2f} F {np.mean(Fg == 0):.2f}")
    assert relf(Wg, Wo) <= 1e-4 and relf(Fg, Fo) <= 1e-4


@pytest.mark.parametrize("flags", [dict(literal_break=1), dict(guard=0), dict(literal_break=1, guard=0)])
def test_ablation_step_parity(flags):
    """The paper-literal inner loop (signed break test, no descent guard, or both): one
    F-half and one W-half each from an identical state, GPU vs oracle, row by row.  Without
    the guard a Newton step can overshoot (to exactly 0, leaving a nonzero with model value
    0 when the break test is signed too), and the next steps start from where it landed, so a
    float32 difference in one step carries into the rest of the coordinate's sequence: rows
    are then held to 1e-5 except for at most 1% of them."""
    prob = CASES["corpus_mid"]()
    t = 2
    ids = oracle.permutation(0, t, 0, prob.r)
    prm = oracle.params(**flags)
    Fo, _, _ = oracle.sweep_F(prob, prob.W0.astype(np.float64), prob.F0.astype(np.float64), ids, prm)
    Fg = gpu_half(prob, prob.W0, prob.F0, t, "F", P.nmfkl_params_default(**flags))
    F1 = Fo.astype(np.float32)
    Wo, _, _ = oracle.sweep_W(prob, F1.astype(np.float64), prob.W0.astype(np.float64), ids, prm)
    Wg = gpu_half(prob, prob.W0, F1, t, "W", P.nmfkl_params_default(**flags))
    res = []
    for name, g, o in (("F", Fg, Fo), ("W", Wg, Wo)):
        rows = np.linalg.norm(g - o, axis=1) / np.maximum(np.linalg.norm(o, axis=1), 1e-300)
        flip = np.any((g == 0) != (o == 0), axis=1)
        print(f"ablation {flags} {name}-half: rel {relf(g, o):.2e}, row max (no flip) "
              f"{rows[~flip].max():.2e}, rows above 1e-5 {int(np.sum(rows > 1e-5))}, rows with a zero flip "
              f"{int(flip.sum())} of {len(rows)}")
        res.append((relf(g, o), rows, flip))
    for rel, rows, flip in res:
        assert rel <= 1e-4
        if flags.get("guard", 1):
            assert rows[~flip].max() <= 1e-5 and flip.sum() <= max(1, len(rows) // 1000)
        else:
            assert np.sum(rows > 1e-5) <= len(rows) // 100


def test_guard_rejections_restore_the_state():
    """With j_max = 0 every decreasing step that fails the descent guard is abandoned at
    once (Alg. 2 with the guard of §3): the lane state must go back to the model before the
    step.  Both halves (the W-half has rows for the long-segment kernels), GPU vs oracle;
    the oracle's counters confirm that rejections happen."""
    prob = CASES["corpus_mid"]()
    t = 2
    ids = oracle.permutation(0, t, 0, prob.r)
    prm = oracle.params(j_max=0)
    Fo, _, st_f = oracle.sweep_F(prob, prob.W0.astype(np.float64), prob.F0.astype(np.float64), ids, prm)
    Wo, _, st_w = oracle.sweep_W(prob, prob.F0.astype(np.float64), prob.W0.astype(np.float64), ids, prm)
    assert st_f["rejects"] > 0 and st_w["rejects"] > 0
    Fg = gpu_half(prob, prob.W0, prob.F0, t, "F", P.nmfkl_params_default(j_max=0))
    Wg = gpu_half(prob, prob.W0, prob.F0, t, "W", P.nmfkl_params_default(j_max=0))
    print(f"j_max = 0: F rel {relf(Fg, Fo):.2e} flips {flips(Fg, Fo)}, W rel {relf(Wg, Wo):.2e} "
          f"flips {flips(Wg, Wo)}; oracle rejections F {st_f['rejects']} W {st_w['rejects']}")
    assert relf(Fg, Fo) <= 1e-4 and relf(Wg, Wo) <= 1e-4


def _bf16_round(a):
    """Round float32 values to the nearest bfloat16 (ties to even), kept as float32."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)


def test_bf16_tiles_exact_when_the_fixed_factor_is_representable():
    """With every fixed-factor entry a bfloat16 value, bf16-stored tiles lose nothing: the
    half-sweep must equal the float32-tile half-sweep up to the summation order of the model
    values (float64 sums of the same exact products: pins the bf16 copy, its column sums,
    the tile loads and the model computed from the tiles)."""
    prob = mid_corpus()
    W = _bf16_round(prob.W0)
    F = _bf16_round(prob.F0)
    for half in ("F", "W"):
        a = gpu_half(prob, W, F, 2, half, P.nmfkl_params_default())
        b = gpu_half(prob, W, F, 2, half, P.nmfkl_params_default(tile_bf16=1))
        e = relf(b, a.astype(np.float64))
        print(f"bf16 tiles on bf16-representable {half}-half input: rel {e:.2e}, flips {flips(a, b)}")
        assert e <= 1e-6, f"{half}-half differs with bf16 tiles"


def test_bf16_tiles_trajectory_error():
    """bf16-stored tiles (float32/float64 arithmetic): the objective stays within 1e-3
    relative of the float32-tile run over 8 sweeps and keeps decreasing."""
    prob = mid_corpus()
    D = {}
    for bf in (0, 1):
        dev = P.upload(prob, "cuda")
        h = P.nmfkl_create(dev, P.nmfkl_params_default(tile_bf16=bf))
        D[bf] = []
        for t in range(8):
            P.nmfkl_sweep_F(h, t)
            P.nmfkl_sweep_W(h, t)
            D[bf].append(P.nmfkl_objective(h))
        P.nmfkl_destroy(h)
    rel = np.abs(np.array(D[1]) - D[0]) / np.array(D[0])
    print(f"bf16 tiles: objective rel diff per sweep {np.array2string(rel, precision=1)}")
    assert rel.max() <= 1e-3
    assert all(D[1][i + 1] <= D[1][i] * (1 + 1e-4) for i in range(7))


def huge_row_problem(m=1_700_000, r=4, seed=0):
    """Row 0 has a nonzero in every column (m nonzeros: more than the co-resident capacity at
    2048 nonzeros per block), row 1 in every 7th column, row 2 in every 11th."""
    g = np.random.default_rng(seed)
    rows, cols = [np.zeros(m, np.int64)], [np.arange(m)]
    for i, step in ((1, 7), (2, 11)):
        c = np.arange(0, m, step)
        rows.append(np.full(c.size, i)); cols.append(c)
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    order = np.lexsort((rows, cols))
    rows, cols = rows[order], cols[order]
    ptr = np.zeros(m + 1, np.int64)
    np.cumsum(np.bincount(cols, minlength=m), out=ptr[1:])
    val = g.geometric(0.6, rows.size).astype(np.float32)
    return workloads._problem(3, m, r, ptr, rows.astype(np.int32), val, seed, 11, {"name": "huge row"})


def test_huge_row_matches_the_oracle():
    prob = huge_row_problem()
    assert np.diff(prob.csr_ptr).max() > 768 * 2048
    t = 0
    ids = oracle.permutation(0, t, 0, prob.r)
    Wo, _, _ = oracle.sweep_W(prob, prob.F0.astype(np.float64), prob.W0.astype(np.float64), ids)
    Wg = gpu_half(prob, prob.W0, prob.F0, t, "W")
    e = relf(Wg, Wo)
    print(f"huge row W-half: rel {e:.2e}; rows {Wg.tolist()}")
    assert e <= 1e-4


def boundary_rows_problem(r=6, seed=0):
    """Rows whose lengths sit on both sides of every length boundary of the W-half's launches:
    the binned variants (32, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 2048), one cooperative
    block (5120), 20 blocks (102,400) and a whole number of the wide blocks (11 x 10,240), plus
    800 rows of 1025..2048 nonzeros (the binned launch's 256 x 8 variant, more of them than a
    256-CU device holds at once)."""
    g = np.random.default_rng(seed)
    edges = [32, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 2048, 5120, 20 * 5120, 11 * 10240]
    lengths = [L for e in edges for L in (e, e + 1)] + list(g.integers(1025, 2049, 800))
    n, m = len(lengths), 11 * 10240 + 1
    rows = np.concatenate([np.full(L, i, np.int64) for i, L in enumerate(lengths)])
    cols = np.concatenate([g.choice(m, L, replace=False) for L in lengths])
    order = np.lexsort((rows, cols))
    rows, cols = rows[order], cols[order]
    ptr = np.zeros(m + 1, np.int64)
    np.cumsum(np.bincount(cols, minlength=m), out=ptr[1:])
    val = g.geometric(0.6, rows.size).astype(np.float32)
    return workloads._problem(n, m, r, ptr, rows.astype(np.int32), val, seed, 12, {"name": "boundary rows"})


def test_every_length_boundary_matches_the_oracle():
    prob = boundary_rows_problem()
    lens = np.diff(prob.csr_ptr)
    assert lens.max() == 11 * 10240 + 1 and ((lens > 1024) & (lens <= 2048)).sum() > 768
    t = 1
    ids = oracle.permutation(0, t, 0, prob.r)
    Wo, _, _ = oracle.sweep_W(prob, prob.F0.astype(np.float64), prob.W0.astype(np.float64), ids)
    Wg = gpu_half(prob, prob.W0, prob.F0, t, "W")
    Fo, _, _ = oracle.sweep_F(prob, prob.W0.astype(np.float64), prob.F0.astype(np.float64), ids)
    Fg = gpu_half(prob, prob.W0, prob.F0, t, "F")
    # each boundary row on its own (the 800 extra rows would hide one wrong row in the norm)
    err = np.linalg.norm(Wg - Wo, axis=1)
    norm = np.linalg.norm(Wo, axis=1)
    nb = 28
    worst = float(np.max(err[:nb] / (norm[:nb] + 1e-5 * norm.max())))
    print(f"boundary rows: W rel {relf(Wg, Wo):.2e} (worst boundary row {worst:.2e}), F rel {relf(Fg, Fo):.2e}")
    assert relf(Wg, Wo) <= 1e-4 and relf(Fg, Fo) <= 1e-4
    assert worst <= 1e-3


def test_queue_of_many_long_rows_matches_the_oracle():
    """300 rows of 8,000-11,000 nonzeros (2-3 cooperating blocks each): more parts than the
    device holds at once, so blocks take parts from the ticket queue as others finish."""
    g = np.random.default_rng(3)
    n, m, r = 300, 24000, 4
    lengths = g.integers(8000, 11001, n)
    rows = np.concatenate([np.full(L, i, np.int64) for i, L in enumerate(lengths)])
    cols = np.concatenate([g.choice(m, L, replace=False) for L in lengths])
    order = np.lexsort((rows, cols))
    rows, cols = rows[order], cols[order]
    ptr = np.zeros(m + 1, np.int64)
    np.cumsum(np.bincount(cols, minlength=m), out=ptr[1:])
    val = g.geometric(0.6, rows.size).astype(np.float32)
    prob = workloads._problem(n, m, r, ptr, rows.astype(np.int32), val, 3, 13, {"name": "queue rows"})
    parts = int(np.sum((lengths + 5119) // 5120))
    assert parts > 2 * 256
    W, F = prob.W0.astype(np.float64), prob.F0.astype(np.float64)
    dev = P.upload(prob, "cuda")
    h = P.nmfkl_create(dev, P.nmfkl_params_default())
    for t in range(2):
        ids = oracle.permutation(0, t, 0, r)
        F, _, _ = oracle.sweep_F(prob, W, F, ids)
        W, _, _ = oracle.sweep_W(prob, F, W, ids)
        P.nmfkl_sweep_F(h, t)
        P.nmfkl_sweep_W(h, t)
    Wg, Fg = dev.W.cpu().numpy(), dev.F.cpu().numpy()
    P.nmfkl_destroy(h)
    print(f"queue rows ({parts} parts): W rel {relf(Wg, W):.2e}, F rel {relf(Fg, F):.2e}")
    assert relf(Wg, W) <= 1e-4 and relf(Fg, F) <= 1e-4


def test_queue_of_many_waves_matches_the_oracle():
    """1,900 rows of 8,000-11,000 nonzeros: a queue of more than 8 waves of the co-resident
    capacity, which runs on the wide blocks (512 threads, 10,240 nonzeros each).  Every row
    is checked on its own, and a second run gives the same factors bit for bit (partners'
    sums are added in part order, whatever order the blocks arrive in)."""
    import torch
    g = np.random.default_rng(5)
    n, m, r = 1900, 24000, 4
    lengths = g.integers(8000, 11001, n)
    rows = np.concatenate([np.full(L, i, np.int64) for i, L in enumerate(lengths)])
    cols = np.concatenate([g.choice(m, L, replace=False) for L in lengths])
    order = np.lexsort((rows, cols))
    rows, cols = rows[order], cols[order]
    ptr = np.zeros(m + 1, np.int64)
    np.cumsum(np.bincount(cols, minlength=m), out=ptr[1:])
    val = g.geometric(0.6, rows.size).astype(np.float32)
    prob = workloads._problem(n, m, r, ptr, rows.astype(np.int32), val, 5, 14, {"name": "many-wave queue"})
    parts = int(np.sum((lengths + 5119) // 5120))
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    assert parts > 8 * 2 * ncu
    t = 2
    ids = oracle.permutation(0, t, 0, r)
    Wo, _, _ = oracle.sweep_W(prob, prob.F0.astype(np.float64), prob.W0.astype(np.float64), ids)
    Wg = gpu_half(prob, prob.W0, prob.F0, t, "W")
    err = np.linalg.norm(Wg - Wo, axis=1) / (np.linalg.norm(Wo, axis=1) + 1e-5 * np.abs(Wo).max())
    print(f"many-wave queue ({parts} parts of 5120): W rel {relf(Wg, Wo):.2e}, worst row {err.max():.2e}")
    assert relf(Wg, Wo) <= 1e-4 and err.max() <= 1e-3
    assert np.array_equal(gpu_half(prob, prob.W0, prob.F0, t, "W"), Wg)
