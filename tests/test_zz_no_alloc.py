"""nmfkl_foldin_noalloc (the fold-in entry point that allocates nothing) against nmfkl_foldin,
through the C ABI on an MI355X: two calls in a row, the second with fewer documents, bit for
bit, plus its device-side rejections."""
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


def _docs(ptr, idx, val):
    import torch
    return torch.from_numpy(ptr).cuda(), torch.from_numpy(idx).cuda(), torch.from_numpy(val).cuda()


def _outputs(nd, r):
    import torch
    return (torch.full((nd, r), -1.0, dtype=torch.float32, device="cuda"),
            torch.full((nd,), -1, dtype=torch.int32, device="cuda"),
            torch.full((nd,), -1.0, dtype=torch.float64, device="cuda"))


def _subset(ptr, idx, val, docs):
    lens = np.diff(ptr)[docs]
    sp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    si = np.concatenate([idx[ptr[d]:ptr[d + 1]] for d in docs]).astype(np.int32)
    sv = np.concatenate([val[ptr[d]:ptr[d + 1]] for d in docs]).astype(np.float32)
    return sp, si, sv


def test_noalloc_foldin_equals_plain_foldin_on_two_calls():
    import torch
    n, r = 6000, 32
    W = workloads.serving_model(n=n, r=r, seed=11)
    _, ptr, idx, val = workloads.serving_requests(700, n=n, seed=12, median_len=80, max_len=5000)
    print(f"noalloc: call 1 of {len(ptr) - 1} documents, longest {np.diff(ptr).max()} words", flush=True)
    Wd = torch.from_numpy(W).cuda()
    m = P.nmfkl_model_create(Wd)
    try:
        d1 = _docs(ptr, idx, val)
        Fa, pa, ka = P.nmfkl_foldin(m, *d1)
        Fb, pb, kb = P.nmfkl_foldin_noalloc(m, *d1, *_outputs(len(ptr) - 1, r))
        assert torch.equal(Fa, Fb) and torch.equal(pa, pb) and torch.equal(ka, kb)
        # second call: fewer documents, in another order, over the scratch the first call left
        docs = np.random.default_rng(5).permutation(len(ptr) - 1)[:123]
        sp, si, sv = _subset(ptr, idx, val, docs)
        print(f"noalloc: call 2 of {len(sp) - 1} documents", flush=True)
        d2 = _docs(sp, si, sv)
        Fc, pc, kc = P.nmfkl_foldin(m, *d2)
        Fd, pd, kd = P.nmfkl_foldin_noalloc(m, *d2, *_outputs(len(sp) - 1, r))
        assert torch.equal(Fc, Fd) and torch.equal(pc, pd) and torch.equal(kc, kd)
        # each document is independent of the others in its call
        assert torch.equal(Fd, Fb[torch.from_numpy(docs).cuda()])
        # and the second call against the oracle (fold-in reading of Alg. 1's F-half)
        Fo, po, ko, _ = oracle.foldin(W, sp, si, sv)
        Fg, pg, kg = Fd.cpu().numpy(), pd.cpu().numpy(), kd.cpu().numpy()
        same = pg == po
        assert same.mean() >= 0.95 and np.all(np.abs(pg - po) <= 1)
        rel = np.linalg.norm(Fg[same] - Fo[same]) / np.linalg.norm(Fo[same])
        assert rel <= 1e-4
        assert np.max(np.abs(kg - ko) / ko) <= 1e-5
    finally:
        P.nmfkl_model_destroy(m)


def test_noalloc_foldin_rejections():
    import torch
    n, r = 6000, 16
    W = workloads.serving_model(n=n, r=r, seed=13)
    Wd = torch.from_numpy(W).cuda()
    m = P.nmfkl_model_create(Wd)
    try:
        # above the scratch's document limit: refused on the host
        big = torch.zeros(16386, dtype=torch.int64, device="cuda")
        with pytest.raises(P.NmfklError) as e:
            P.nmfkl_foldin_noalloc(m, big, torch.zeros(1, dtype=torch.int32, device="cuda"),
                                   torch.zeros(1, dtype=torch.float32, device="cuda"), *_outputs(16385, r))
        assert e.value.code == -6
        # pointers not monotone: refused by the device check before any fold-in kernel
        ptr = np.array([0, 3, 2, 5], np.int64)
        idx = np.array([1, 2, 3, 4, 5], np.int32)
        val = np.ones(5, np.float32)
        with pytest.raises(P.NmfklError) as e:
            P.nmfkl_foldin_noalloc(m, *_docs(ptr, idx, val), *_outputs(3, r))
        assert e.value.code == -1
        # a word id out of range
        ptr = np.array([0, 2, 5], np.int64)
        idx = np.array([1, 2, 3, 4, n], np.int32)
        with pytest.raises(P.NmfklError) as e:
            P.nmfkl_foldin_noalloc(m, *_docs(ptr, idx, val), *_outputs(2, r))
        assert e.value.code == -1
        # a document above the largest fold-in variant
        L = 5121
        ptr = np.array([0, 2, 2 + L], np.int64)
        idx = np.concatenate([[0, 1], np.arange(L)]).astype(np.int32)
        val = np.ones(L + 2, np.float32)
        with pytest.raises(P.NmfklError) as e:
            P.nmfkl_foldin_noalloc(m, *_docs(ptr, idx, val), *_outputs(2, r))
        assert e.value.code == -6
        # after the refusals a valid call still works and matches the plain entry point
        ptr = np.array([0, 2, 5], np.int64)
        idx = np.array([1, 2, 3, 4, 5], np.int32)
        val = np.array([1, 2, 3, 1, 4], np.float32)
        d = _docs(ptr, idx, val)
        Fa, pa, ka = P.nmfkl_foldin(m, *d)
        Fb, pb, kb = P.nmfkl_foldin_noalloc(m, *d, *_outputs(2, r))
        assert torch.equal(Fa, Fb) and torch.equal(pa, pb) and torch.equal(ka, kb)
    finally:
        P.nmfkl_model_destroy(m)
