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


def _slow_and_fast(W, seed=21):
    """One document of 5,000 distinct words (many passes over a 512-lane block) and 50 of one
    word (one or two passes each)."""
    n = W.shape[0]
    g = np.random.default_rng(seed)
    slow = (np.sort(g.choice(n, 5000, replace=False)).astype(np.int32),
            (1 + g.geometric(0.3, 5000)).astype(np.float32))
    fast = [(np.array([w], np.int32), np.array([3.0], np.float32)) for w in g.choice(n, 50, replace=False)]
    return slow, fast


def _drain(srv, want, limit=60.0):
    out, polls = {}, []
    t0 = time.time()
    while len(out) < want:
        got = P.nmfkl_server_poll(srv, 1024)
        if got:
            polls.append([rec[0] for rec in got])
        for rec in got:
            out[rec[0]] = rec
        assert time.time() - t0 < limit
    return out, polls


def test_server_returns_each_document_when_it_finishes(small_serving):
    """One lane runs one batch: the slow document and 50 one-word documents.  The one-word
    documents come back before the slow one, in earlier polls, while the lane still runs."""
    import torch
    W = small_serving[0]
    m = P.nmfkl_model_create(torch.from_numpy(W).cuda())
    srv = P.nmfkl_server_create(m, 64 << 20, lanes=1, lane_docs=64)
    slow, fast = _slow_and_fast(W)
    assert P.nmfkl_server_submit(srv, 1000, *slow) == 0
    for k, d in enumerate(fast):
        assert P.nmfkl_server_submit(srv, k, *d) == 0
    out, polls = _drain(srv, 51)
    assert all(rec[6] == 0 for rec in out.values())
    assert 1000 not in polls[0], "the slow document came back with the first results"
    assert max(out[k][4] for k in range(50)) < out[1000][4]
    print(f"per-document return: {len(polls)} polls returned results; slow document {out[1000][1]} passes, "
          f"{(out[1000][4] - max(out[k][4] for k in range(50))) * 1e3:.2f} ms after the last one-word document")
    # and each result equals plain fold-in of the same document
    dp = torch.tensor([0, slow[0].size], dtype=torch.int64, device="cuda")
    F, ps, kl = P.nmfkl_foldin(m, dp, torch.from_numpy(slow[0]).cuda(), torch.from_numpy(slow[1]).cuda())
    assert np.array_equal(F.cpu().numpy()[0], out[1000][5]) and int(ps[0]) == out[1000][1]
    P.nmfkl_server_destroy(srv)
    P.nmfkl_model_destroy(m)


def test_server_timeout_cancel_and_busy(small_serving):
    """With the single lane busy: a document whose time limit passes while it waits comes back
    expired, before the lane frees; a waiting document can be cancelled, a launched one cannot; the waiting queue
    refuses documents beyond max_queued with NMFKL_E_BUSY."""
    import torch
    W = small_serving[0]
    m = P.nmfkl_model_create(torch.from_numpy(W).cuda())
    srv = P.nmfkl_server_create(m, 64 << 20, lanes=1, lane_docs=64, max_queued=3)
    slow, fast = _slow_and_fast(W, seed=22)
    assert P.nmfkl_server_submit(srv, 1000, *slow) == 0
    assert P.nmfkl_server_poll(srv, 0) == []              # launches the slow document
    assert P.nmfkl_server_submit(srv, 1, *fast[0], timeout_s=1e-6) == 0
    assert P.nmfkl_server_submit(srv, 2, *fast[1]) == 0
    assert P.nmfkl_server_submit(srv, 3, *fast[2]) == 0
    assert P.nmfkl_server_submit(srv, 4, *fast[3]) == -5     # three are waiting: busy
    assert P.nmfkl_server_cancel(srv, 2) == 0
    assert P.nmfkl_server_cancel(srv, 2) == -1               # already withdrawn
    assert P.nmfkl_server_cancel(srv, 1000) == -1            # launched: runs to the end
    assert P.nmfkl_server_submit(srv, 4, *fast[3]) == 0      # a slot is free again
    out, polls = _drain(srv, 5)
    assert out[1000][6] == 0 and out[3][6] == 0 and out[4][6] == 0
    assert out[1][6] == P.RESULT_EXPIRED and out[1][1] == 0
    # the expired document is returned while the slow one still holds the lane
    first = {i: min(k for k, p in enumerate(polls) if i in p) for i in (1, 1000)}
    assert first[1] < first[1000], polls
    assert out[2][6] == P.RESULT_CANCELLED and out[2][1] == 0
    # the words of launched documents are released once their lane is free again
    t0 = time.time()
    while P.nmfkl_server_pending(srv) != (0, 0):
        assert P.nmfkl_server_poll(srv, 8) == []
        assert time.time() - t0 < 10
    P.nmfkl_server_destroy(srv)
    P.nmfkl_model_destroy(m)
