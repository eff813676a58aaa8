"""Batched problems on the GPU, through the C ABI (need an MI355X).

A batch advances many independent problems with shared launches captured in a graph.  Each
problem's arithmetic is that of a handle over the same problem with the same parameters, so
the factors must agree bit for bit with solo handles running the same sweeps; the solo path
is checked against the FP64 oracle in test_gpu_parity.py, and every batch member is checked
against the oracle here directly.
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


def _corpus(n, m, r, seed, tag):
    ptr, idx, val = workloads.corpus(n, m, 80.0, 1.0, 2000, 1.1, 0.6, seed=seed, tag=tag)
    return workloads._problem(n, m, r, ptr, idx, val, seed, tag, {"name": f"corpus {n}x{m} r={r}"})


@pytest.fixture(scope="module")
def problems():
    """Uneven shapes, ranks 10..64, one with rows long enough for cooperative launches."""
    probs = workloads.batched_configs(seed=3, count=6, scale=0.06)
    probs.append(workloads.config(0, seed=0))                 # tiny 500 x 400, r = 10
    probs.append(_corpus(2000, 20000, 12, seed=0, tag=8))     # rows up to ~20k nonzeros
    probs.append(_corpus(1500, 3000, 64, seed=1, tag=9))
    lens = np.concatenate([np.diff(p.csr_ptr) for p in probs])
    assert lens.max() > 2 * 2048 and ((lens > 1024) & (lens <= 2048)).any()
    return probs


def solo(prob, t0, nsweeps, prm):
    dev = P.upload(prob, "cuda")
    h = P.nmfkl_create(dev, prm)
    for t in range(t0, t0 + nsweeps):
        P.nmfkl_sweep_F(h, t)
        P.nmfkl_sweep_W(h, t)
    D = P.nmfkl_objective_carried(h)
    W, F = dev.W.cpu().numpy(), dev.F.cpu().numpy()
    P.nmfkl_destroy(h)
    return W, F, D


def test_batch_equals_solo_bitwise_and_graph_replays(problems):
    prm = P.nmfkl_params_default()
    devs = [P.upload(p, "cuda") for p in problems]
    b = P.nmfkl_batch_create(devs, prm)
    # two graph launches of the same captured graph with different t0 (t from device memory)
    P.nmfkl_batch_run(b, 0, 2)
    P.nmfkl_batch_run(b, 2, 2)
    D = P.nmfkl_batch_objective(b)
    info = P.nmfkl_batch_get_info(b)
    print("batch info", info)
    assert info["nprob"] == len(problems) and info["graph_cooperative"] in (0, 1)
    assert info["long_rounds"][1] == 1 and info["long_parts"][1] >= 2
    for q, p in enumerate(problems):
        W, F, Ds = solo(p, 0, 4, prm)
        Wb, Fb = devs[q].W.cpu().numpy(), devs[q].F.cpu().numpy()
        assert np.array_equal(W, Wb), f"problem {q}: W differs"
        assert np.array_equal(F, Fb), f"problem {q}: F differs"
        assert D[q] == Ds, f"problem {q}: D {D[q]} vs {Ds}"
    P.nmfkl_batch_destroy(b)


def test_batch_members_vs_oracle(problems):
    """Every member of the batch (ranks 10..64, uneven shapes, rows long enough for the
    cooperative launches) against the oracle's own run: objective after each of 6 sweeps
    within 1e-5, factors within 1e-4 relative Frobenius, and at most 1% of rows above 1e-3."""
    devs = [P.upload(p, "cuda") for p in problems]
    b = P.nmfkl_batch_create(devs)
    state = [(p.W0.astype(np.float64), p.F0.astype(np.float64)) for p in problems]
    worst = np.zeros(len(problems))
    for t in range(6):
        P.nmfkl_batch_run(b, t, 1)
        Dg = P.nmfkl_batch_objective(b)
        for q, prob in enumerate(problems):
            W, F = state[q]
            ids = oracle.permutation(0, t, 0, prob.r)
            F, _, _ = oracle.sweep_F(prob, W, F, ids)
            W, _, _ = oracle.sweep_W(prob, F, W, ids)
            state[q] = (W, F)
            Do = oracle.objective(prob, W, F)
            worst[q] = max(worst[q], abs(Dg[q] - Do) / Do)
    for q, prob in enumerate(problems):
        W, F = state[q]
        Wg, Fg = devs[q].W.cpu().numpy().astype(np.float64), devs[q].F.cpu().numpy().astype(np.float64)
        eW = float(np.linalg.norm(Wg - W) / np.linalg.norm(W))
        eF = float(np.linalg.norm(Fg - F) / np.linalg.norm(F))
        rows = np.linalg.norm(Wg - W, axis=1) / np.maximum(np.linalg.norm(W, axis=1), 1e-300)
        print(f"member {q} ({prob.n}x{prob.m}, r={prob.r}, nnz {prob.nnz}): D rel max {worst[q]:.1e}, "
              f"W {eW:.2e} F {eF:.2e}, W rows above 1e-3 {int(np.sum(rows > 1e-3))}")
        assert worst[q] <= 1e-5 and eW <= 1e-4 and eF <= 1e-4
        assert np.sum(rows > 1e-3) <= max(1, len(rows) // 100)
    P.nmfkl_batch_destroy(b)


def test_tuner_restores_state_and_solo_reproduces_choice(problems):
    devs = [P.upload(p, "cuda") for p in problems]
    b = P.nmfkl_batch_create(devs)
    P.nmfkl_batch_run(b, 0, 1)
    before = [(d.W.cpu().numpy(), d.F.cpu().numpy()) for d in devs]
    chosen = P.nmfkl_batch_tune(b, 1)
    print(f"tuner chose bin_shift={chosen.bin_shift} tuning={chosen.tuning}")
    for q, d in enumerate(devs):
        assert np.array_equal(before[q][0], d.W.cpu().numpy()), f"problem {q}: W changed by the tuner"
        assert np.array_equal(before[q][1], d.F.cpu().numpy()), f"problem {q}: F changed by the tuner"
    info = P.nmfkl_batch_get_info(b)
    assert info["bin_shift"] == chosen.bin_shift and info["tuning"] == chosen.tuning
    P.nmfkl_batch_run(b, 1, 2)
    D = P.nmfkl_batch_objective(b)
    for q in (0, 6, 7):
        W, F, Ds = solo(problems[q], 0, 3, chosen)
        assert np.array_equal(W, devs[q].W.cpu().numpy()), f"problem {q}: W differs"
        assert np.array_equal(F, devs[q].F.cpu().numpy()), f"problem {q}: F differs"
        assert D[q] == Ds
    P.nmfkl_batch_destroy(b)


@pytest.mark.parametrize("shift", [1, 2])
def test_bin_shift_changes_rounding_only(shift):
    """Another lane mapping sums in another order: results stay within the oracle tolerance."""
    prob = workloads.config(0, seed=1, n=3000, m=2500, r=16, density=0.01)
    W0, F0, D0 = solo(prob, 0, 3, P.nmfkl_params_default())
    W1, F1, D1 = solo(prob, 0, 3, P.nmfkl_params_default(bin_shift=shift))
    e = float(np.linalg.norm(F1.astype(np.float64) - F0) / np.linalg.norm(F0))
    print(f"bin_shift {shift}: F rel {e:.2e}, D rel {abs(D1 - D0) / D0:.2e}")
    assert abs(D1 - D0) / D0 <= 1e-5 and e <= 1e-4


def test_batch_create_rejects_bad_problem(problems):
    import torch
    devs = [P.upload(p, "cuda") for p in problems[:2]]
    devs[1].W[0, 0] = float("nan")
    torch.cuda.synchronize()
    with pytest.raises(P.NmfklError) as ei:
        P.nmfkl_batch_create(devs)
    assert ei.value.code == -1 and "problem 1" in ei.value.message
