"""Fold-in and the continuously batched server, through the C ABI (MI355X)."""
import time

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


@pytest.fixture(scope="module")
def small_serving():
    n, r = 6000, 32
    W = workloads.serving_model(n=n, r=r, seed=3)
    _, ptr, idx, val = workloads.serving_requests(600, n=n, seed=4, median_len=80, max_len=2000)
    return W, ptr, idx, val


def device_docs(ptr, idx, val):
    import torch
    return (torch.from_numpy(ptr).cuda(), torch.from_numpy(idx).cuda(), torch.from_numpy(val).cuda())


def test_foldin_parity_with_oracle(small_serving):
    import torch
    W, ptr, idx, val = small_serving
    Wd = torch.from_numpy(W).cuda()
    m = P.nmfkl_model_create(Wd)
    F, passes, kl = P.nmfkl_foldin(m, *device_docs(ptr, idx, val))
    Fg, pg, kg = F.cpu().numpy(), passes.cpu().numpy(), kl.cpu().numpy()
    P.nmfkl_model_destroy(m)
    Fo, po, ko, _ = oracle.foldin(W, ptr, idx, val)
    same = pg == po
    print(f"fold-in: passes equal for {same.mean():.3f} of docs (median {np.median(po)}, max {po.max()}); "
          f"F rel {relf(Fg[same], Fo[same]):.2e} (equal passes), all {relf(Fg, Fo):.2e}; "
          f"KL rel max {np.max(np.abs(kg - ko) / ko):.2e}")
    assert same.mean() >= 0.95 and np.all(np.abs(pg - po) <= 1)
    assert relf(Fg[same], Fo[same]) <= 1e-4
    assert np.max(np.abs(kg - ko) / ko) <= 1e-5
    assert np.all(Fg >= 0)


def test_server_matches_plain_and_is_independent_of_the_mix(small_serving):
    import torch
    W, ptr, idx, val = small_serving
    Wd = torch.from_numpy(W).cuda()
    m = P.nmfkl_model_create(Wd)
    F, passes, kl = P.nmfkl_foldin(m, *device_docs(ptr, idx, val))
    Fp = F.cpu().numpy()
    nd = len(ptr) - 1
    srv = P.nmfkl_server_create(m, 64 << 20, lanes=4, lane_docs=64)
    doc = lambda d: (idx[ptr[d]:ptr[d + 1]], val[ptr[d]:ptr[d + 1]])

    def run(ids):
        for d in ids:
            while P.nmfkl_server_submit(srv, d, *doc(d)) != 0:
                P.nmfkl_server_poll(srv, 0)
        out = {}
        t0 = time.time()
        while len(out) < len(ids):
            for rec in P.nmfkl_server_poll(srv, 1024):
                out[rec[0]] = rec
            assert time.time() - t0 < 120
        return out

    alone = run([7])
    mix = run(list(range(nd)))
    assert np.array_equal(alone[7][5], mix[7][5])            # same document alone and in the mix
    Fs = np.stack([mix[d][5] for d in range(nd)])
    assert np.array_equal(Fs, Fp)                            # server == plain fold-in, bit for bit
    assert all(mix[d][1] == int(passes[d]) for d in range(nd))
    lat = np.array([rec[4] - rec[3] for rec in mix.values()])
    assert np.all(lat >= 0)
    P.nmfkl_server_destroy(srv)
    P.nmfkl_model_destroy(m)


def test_server_admission_by_memory(small_serving):
    import torch
    W, ptr, idx, val = small_serving
    m = P.nmfkl_model_create(torch.from_numpy(W).cuda())
    budget = 5120 * 8  # exactly one largest document
    srv = P.nmfkl_server_create(m, budget, lanes=1, lane_docs=8)
    big = np.arange(0, 5120, dtype=np.int32)
    ones = np.ones(big.size, np.float32)
    assert P.nmfkl_server_submit(srv, 1, big, ones) == 0
    assert P.nmfkl_server_submit(srv, 2, big[:100], ones[:100]) == -2    # refused: budget full
    got = []
    t0 = time.time()
    while not got:
        got = P.nmfkl_server_poll(srv, 8)
        assert time.time() - t0 < 60
    assert P.nmfkl_server_submit(srv, 2, big[:100], ones[:100]) == 0     # admitted after completion
    with pytest.raises(P.NmfklError):
        P.nmfkl_server_submit(srv, 3, np.array([5, 3], np.int32), np.ones(2, np.float32))  # not increasing
    P.nmfkl_server_destroy(srv)
    P.nmfkl_model_destroy(m)


def test_long_documents_vs_oracle(small_serving):
    """Documents of 2049..5120 distinct words (one document per 256- or 512-lane block)."""
    import torch
    W, _, _, _ = small_serving
    n = W.shape[0]
    g = np.random.default_rng(11)
    lens = [1500, 2049, 3000, 4100, 5000, 5120]
    idx = [np.sort(g.choice(n, L, replace=False)).astype(np.int32) for L in lens]
    val = [(1 + g.geometric(0.6, L) - 1).astype(np.float32) for L in lens]
    ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    idx, val = np.concatenate(idx), np.concatenate(val)
    m = P.nmfkl_model_create(torch.from_numpy(W).cuda())
    F, passes, kl = P.nmfkl_foldin(m, *device_docs(ptr, idx, val))
    Fg, pg, kg = F.cpu().numpy(), passes.cpu().numpy(), kl.cpu().numpy()
    P.nmfkl_model_destroy(m)
    Fo, po, ko, _ = oracle.foldin(W, ptr, idx, val)
    same = pg == po
    print(f"long docs: passes gpu {pg.tolist()} oracle {po.tolist()}; F rel {relf(Fg[same], Fo[same]):.2e}; "
          f"KL rel max {np.max(np.abs(kg - ko) / ko):.2e}")
    assert np.all(np.abs(pg - po) <= 1) and same.sum() >= len(lens) - 1
    assert relf(Fg[same], Fo[same]) <= 1e-4
    assert np.max(np.abs(kg - ko) / ko) <= 1e-5
    too_long = np.arange(5121, dtype=np.int32)
    srv = P.nmfkl_server_create(P.nmfkl_model_create(torch.from_numpy(W).cuda()), 1 << 20)
    with pytest.raises(P.NmfklError) as ei:
        P.nmfkl_server_submit(srv, 1, too_long, np.ones(too_long.size, np.float32))
    assert ei.value.code == -6
