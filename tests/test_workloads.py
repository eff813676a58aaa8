"""Synthetic inputs: structure and the stated distributions."""
import math

import numpy as np

from paper_1604_04026_amd import workloads


def _check_structure(p):
    assert p.csc_ptr.dtype == np.int64 and p.csc_idx.dtype == np.int32 and p.csc_val.dtype == np.float32
    assert p.csc_ptr[0] == 0 and np.all(np.diff(p.csc_ptr) >= 0) and p.csc_ptr[-1] == p.nnz
    assert p.csr_ptr[-1] == p.nnz
    for j in range(0, p.m, max(1, p.m // 200)):
        seg = p.csc_idx[p.csc_ptr[j]:p.csc_ptr[j + 1]]
        assert np.all(np.diff(seg) > 0) and (seg.size == 0 or (seg[0] >= 0 and seg[-1] < p.n))
    # CSR is the transpose of CSC
    rows = np.repeat(np.arange(p.n), np.diff(p.csr_ptr))
    cols = np.repeat(np.arange(p.m), np.diff(p.csc_ptr))
    a = np.lexsort((p.csc_idx, cols))
    key_csc = np.sort(cols.astype(np.int64) * p.n + p.csc_idx)
    key_csr = np.sort(p.csr_idx.astype(np.int64) * p.n + rows)
    assert np.array_equal(key_csc, key_csr)
    assert np.all(p.csc_val > 0) and np.all(np.isfinite(p.csc_val))
    assert p.W0.shape == (p.n, p.r) and p.F0.shape == (p.m, p.r)
    assert p.W0.min() >= 0 and p.W0.max() < 1


def test_planted_tiny():
    p = workloads.config(0)
    _check_structure(p)
    assert abs(p.nnz / (p.n * p.m) - 0.02) < 0.003
    assert (np.diff(p.csc_ptr) == 0).sum() > 0 and (np.diff(p.csr_ptr) == 0).sum() > 0  # empty cols/rows
    assert np.all(p.csc_val == np.round(p.csc_val))


def test_corpus_statistics_small():
    n, m = 5000, 4000
    ptr, idx, val = workloads.corpus(n, m, 80.0, 1.0, 2000, 1.1, 0.6, seed=3)
    L = np.diff(ptr)
    assert 1 <= L.min() and L.max() <= 2000
    assert abs(np.median(L) - 80) < 8
    assert abs(np.log(L).std() - 1.0) < 0.08
    assert abs(val.mean() - 1 / 0.6) < 0.03
    cnt = np.bincount(idx, minlength=n)
    # Zipf head: the most frequent word appears in most documents
    assert cnt.max() > 0.8 * m
    for j in range(0, m, 97):
        seg = idx[ptr[j]:ptr[j + 1]]
        assert np.all(np.diff(seg) > 0)


def test_generation_is_deterministic():
    a = workloads.config(0, seed=5)
    b = workloads.config(0, seed=5)
    assert np.array_equal(a.csc_idx, b.csc_idx) and np.array_equal(a.W0, b.W0)
    c = workloads.config(0, seed=6)
    assert not np.array_equal(a.W0, c.W0)


def test_parallel_generation_is_identical():
    """Document blocks carry their own seeds: forked workers give the same corpus, and the
    batched members are the same whether generated serially or in workers."""
    a = workloads.corpus(1500, 24000, 80.0, 1.0, 2000, 1.1, 0.6, seed=3, tag=5, doc_block=5000)
    b = workloads.corpus(1500, 24000, 80.0, 1.0, 2000, 1.1, 0.6, seed=3, tag=5, doc_block=5000, workers=3)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    p = workloads.batched_configs(seed=1, count=3, scale=0.05)
    q = workloads.batched_configs(seed=1, count=3, scale=0.05, workers=3)
    for x, y in zip(p, q):
        assert np.array_equal(x.csc_idx, y.csc_idx) and np.array_equal(x.csr_val, y.csr_val)
        assert np.array_equal(x.W0, y.W0) and np.array_equal(x.F0, y.F0)
