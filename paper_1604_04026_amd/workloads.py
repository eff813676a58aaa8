"""Seeded synthetic inputs shaped like the paper's sparse count corpora.

The paper evaluates on four downloaded corpora (its Table 1: Digits, Reuters21578,
TDT2, RCV1_4Class).  None of them is available here, so every workload is drawn from a
seeded generator with the shapes, sparsity and value distributions of sparse
document-term count data:

* ``planted``  -- V = Poisson(c * W*^T F*) with Gamma(0.1, 1) factors of rank r*, the
  scale c calibrated so that the expected density hits a target (tiny and batched cases);
* ``corpus``   -- document-like counts: log-normal document lengths, bounded Zipf word
  ids drawn without repetition inside a document, counts 1 + Geometric (the
  document-corpus cases);
* ``requests`` -- a Poisson-arriving stream of single documents for fold-in serving.

This module holds none of the factorisation arithmetic: it only produces V (as CSC and
CSR copies), the uniform(0, 1) initial factors and the serving stream.  It is the one
module shared by the GPU path's tests and by the CPU oracle's tests.

Layout conventions (used by every consumer):
  V is n x m (n = vocabulary / instance dimension, m = documents / instances).
  CSC: ptr int64[m+1], idx int32[nnz] (row ids, strictly increasing per column),
       val float32[nnz].
  CSR: ptr int64[n+1], idx int32[nnz] (column ids, strictly increasing per row),
       val float32[nnz].
  Factors are stored point-major: W as n x r, F as m x r (row-major float32), i.e. the
  paper's W (r x n) and F (r x m) transposed, one contiguous r-vector per word/document.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Problem", "planted", "corpus", "uniform_init", "csc_to_csr", "config",
    "batched_configs", "serving_model", "serving_requests", "CONFIG_NAMES",
]

CONFIG_NAMES = {
    0: "tiny planted 500x400 r=10",
    1: "doc-like corpus 50000x100000 r=50",
    2: "large corpus 100000x2000000 r=100",
    3: "batched 64 planted problems",
    4: "serving fold-in W 50000x100",
}


@dataclasses.dataclass
class Problem:
    n: int
    m: int
    r: int
    csc_ptr: np.ndarray
    csc_idx: np.ndarray
    csc_val: np.ndarray
    csr_ptr: np.ndarray
    csr_idx: np.ndarray
    csr_val: np.ndarray
    W0: np.ndarray
    F0: np.ndarray
    meta: dict

    @property
    def nnz(self) -> int:
        return int(self.csc_ptr[-1])


def _rng(*words: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(w) for w in words]))


def csc_to_csr(n: int, m: int, ptr: np.ndarray, idx: np.ndarray, val: np.ndarray):
    """Structural transpose of a CSC matrix (rows sorted per column) into CSR."""
    nnz = int(ptr[-1])
    cols = np.repeat(np.arange(m, dtype=np.int32), np.diff(ptr).astype(np.int64))
    order = np.argsort(idx, kind="stable")          # stable: columns stay increasing
    rptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(idx, minlength=n), out=rptr[1:])
    assert rptr[-1] == nnz
    return rptr, cols[order].astype(np.int32), val[order].astype(np.float32)


def _from_triplets(n: int, m: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray):
    """CSC from (row, col, val) triplets with unique (row, col) pairs."""
    order = np.lexsort((rows, cols))
    rows, cols, vals = rows[order], cols[order], vals[order]
    ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(cols, minlength=m), out=ptr[1:])
    return ptr, rows.astype(np.int32), vals.astype(np.float32)


def uniform_init(n: int, m: int, r: int, seed: int, tag: int = 0):
    """Random initial factors (the paper leaves the distribution open): iid uniform(0,1)."""
    g = _rng(0x1417, tag, seed)
    W0 = g.random((n, r), dtype=np.float32)
    F0 = g.random((m, r), dtype=np.float32)
    return W0, F0


def planted(n: int, m: int, r_star: int, density: float, seed: int, tag: int = 0):
    """V = Poisson(c * W*^T F*), W* (r* x n), F* (r* x m) iid Gamma(shape 0.1, scale 1).

    The scale c is found by bisection so that the expected fraction of nonzero cells,
    mean(1 - exp(-c M)), equals ``density`` (over all cells when n*m <= 4e6, else over a
    seeded sample of 1e6 cells).  The Poisson counts are drawn by superposition: for
    each component k, N_k ~ Poisson(c * sum(W*_k) * sum(F*_k)) events are placed at rows
    ~ W*_k / sum(W*_k) and columns ~ F*_k / sum(F*_k); events in the same cell add up.
    This has exactly the distribution of cellwise Poisson(c * (W*^T F*)_ij) draws.
    Returns (csc_ptr, csc_idx, csc_val, W*, F*, c).
    """
    g = _rng(0x51A7, tag, seed)
    Ws = g.gamma(0.1, 1.0, size=(r_star, n))
    Fs = g.gamma(0.1, 1.0, size=(r_star, m))
    if n * m <= 4_000_000:
        M = (Ws.T @ Fs).ravel()
    else:
        ii = g.integers(0, n, 1_000_000)
        jj = g.integers(0, m, 1_000_000)
        M = np.einsum("ki,ki->i", Ws[:, ii], Fs[:, jj])
    lo, hi = 0.0, 1.0
    while np.mean(-np.expm1(-hi * M)) < density:
        hi *= 2.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if np.mean(-np.expm1(-mid * M)) < density:
            lo = mid
        else:
            hi = mid
    c = 0.5 * (lo + hi)
    rows, cols = [], []
    sw, sf = Ws.sum(axis=1), Fs.sum(axis=1)
    for k in range(r_star):
        Nk = g.poisson(c * sw[k] * sf[k])
        if Nk == 0:
            continue
        rows.append(g.choice(n, Nk, p=Ws[k] / sw[k]))
        cols.append(g.choice(m, Nk, p=Fs[k] / sf[k]))
    rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    cols = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    key = cols.astype(np.int64) * n + rows
    ukey, cnt = np.unique(key, return_counts=True)
    ptr, idx, val = _from_triplets(n, m, (ukey % n).astype(np.int64),
                                   (ukey // n).astype(np.int64), cnt.astype(np.float32))
    return ptr, idx, val, Ws, Fs, c


def _zipf_cdf(n: int, s: float) -> np.ndarray:
    w = np.arange(1, n + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    return cdf / cdf[-1]


def _distinct_draws(lengths: np.ndarray, cdf: np.ndarray, g: np.random.Generator):
    """For each document, the first L distinct word ranks of an iid Zipf draw sequence.

    Returns (doc, rank) pairs (order inside a document arbitrary).  Draws are made in
    rounds; each round extends the draw sequence of every document that still lacks
    distinct words, so the result is exactly "draw until L distinct".
    """
    m = len(lengths)
    n = len(cdf)
    need = lengths.astype(np.int64)
    seq_next = np.zeros(m, dtype=np.int64)
    out_d, out_r = [], []
    kd = np.zeros(0, np.int64)
    kr = np.zeros(0, np.int64)
    ks = np.zeros(0, np.int64)
    active = np.nonzero(need > 0)[0]
    while active.size:
        have = np.bincount(kd, minlength=m)
        k = 2 * (need[active] - have[active]) + 8
        d = np.repeat(active, k)
        seq = np.repeat(seq_next[active], k) + (np.arange(d.size) - np.repeat(np.cumsum(k) - k, k))
        seq_next[active] += k
        rk = np.minimum(np.searchsorted(cdf, g.random(d.size), side="right"), n - 1)
        alld = np.concatenate([kd, d])
        allr = np.concatenate([kr, rk])
        alls = np.concatenate([ks, seq])
        assert alls.max(initial=0) < (1 << 24) and n * m < (1 << 39)
        # first occurrence of each (doc, rank) in draw order: one composite sort key
        order = np.argsort(((alld * n + allr) << 24) | alls)
        alld, allr, alls = alld[order], allr[order], alls[order]
        first = np.ones(alld.size, dtype=bool)
        first[1:] = (alld[1:] != alld[:-1]) | (allr[1:] != allr[:-1])
        alld, allr, alls = alld[first], allr[first], alls[first]
        # keep the L earliest distinct draws of each document
        order = np.argsort((alld << 24) | alls)
        alld, allr, alls = alld[order], allr[order], alls[order]
        start = np.searchsorted(alld, np.arange(m))
        keep = (np.arange(alld.size) - start[alld]) < need[alld]
        alld, allr, alls = alld[keep], allr[keep], alls[keep]
        cnt = np.bincount(alld, minlength=m)
        complete = cnt[alld] >= need[alld]
        out_d.append(alld[complete])
        out_r.append(allr[complete])
        kd, kr, ks = alld[~complete], allr[~complete], alls[~complete]
        active = np.unique(kd)
    return np.concatenate(out_d), np.concatenate(out_r)


def _corpus_block(args):
    lengths, cdf, relabel, seed, tag, b0 = args
    gb = _rng(0xC0DE, tag, seed, b0)
    d, rk = _distinct_draws(lengths, cdf, gb)
    words = relabel[rk]
    order = np.lexsort((words, d))
    return words[order].astype(np.int32)


def corpus(n: int, m: int, median_len: float, sigma: float, max_len: int,
           zipf_s: float, geom_p: float, seed: int, tag: int = 0, doc_block: int = 200_000,
           workers: int = 1, progress=None):
    """Document-like counts V (n words x m documents).

    * distinct words per document L ~ round(LogNormal(ln median_len, sigma)), clipped to
      [1, max_len];
    * word ranks iid bounded Zipf(zipf_s) on {1..n} (inverse CDF), redrawn until L distinct;
    * ranks relabelled to word ids by one seeded random permutation (heavy rows are not
      contiguous);
    * counts 1 + Geometric_0(geom_p), i.e. numpy's geometric(p) on {1, 2, ...}.
    Documents are drawn in blocks of ``doc_block`` with a seed of their own, so ``workers``
    > 1 (forked processes; call before the process uses a GPU) gives the same result.
    Returns (csc_ptr, csc_idx, csc_val).
    """
    g = _rng(0xC0DE, tag, seed)
    lengths = np.clip(np.rint(g.lognormal(math.log(median_len), sigma, m)), 1, max_len).astype(np.int64)
    lengths = np.minimum(lengths, n)
    relabel = g.permutation(n).astype(np.int64)
    cdf = _zipf_cdf(n, zipf_s)
    ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lengths, out=ptr[1:])
    nnz = int(ptr[-1])
    idx = np.empty(nnz, dtype=np.int32)
    blocks = list(range(0, m, doc_block))
    jobs = [(lengths[b0:min(m, b0 + doc_block)], cdf, relabel, seed, tag, b0) for b0 in blocks]
    if workers <= 1 or len(blocks) == 1:
        results = map(_corpus_block, jobs)
        pool = None
    else:
        import concurrent.futures as cf
        import multiprocessing as mp
        pool = cf.ProcessPoolExecutor(max_workers=min(workers, len(blocks)), mp_context=mp.get_context("fork"))
        results = pool.map(_corpus_block, jobs)
    for k, (b0, words) in enumerate(zip(blocks, results)):
        b1 = min(m, b0 + doc_block)
        idx[ptr[b0]:ptr[b1]] = words
        if progress:
            progress(f"documents {b1} of {m} drawn")
    if pool is not None:
        pool.shutdown()
    gv = _rng(0xC0DF, tag, seed)
    val = gv.geometric(geom_p, nnz).astype(np.float32)
    return ptr, idx, val


def _problem(n, m, r, ptr, idx, val, seed, tag, meta) -> Problem:
    rptr, ridx, rval = csc_to_csr(n, m, ptr, idx, val)
    W0, F0 = uniform_init(n, m, r, seed, tag)
    return Problem(n, m, r, ptr, idx, val, rptr, ridx, rval, W0, F0, meta)


def config(i: int, seed: int = 0, **overrides) -> Problem:
    """The named workloads.

    0: tiny planted problem, V 500 x 400, ~2% density, r* = r = 10, 10 sweeps.
    1: document-like corpus, 50,000 words x 100,000 documents, median length 80
       (log-normal sigma 1, cap 2,000), Zipf(1.1) words, 1 + Geometric(0.6) counts,
       r = 50, 20 sweeps.
    2: large corpus, 100,000 x 2,000,000, log-normal mean ~150 (median 92, sigma 1,
       cap 2,000), r = 100, 10 sweeps.
    ``overrides`` may shrink n, m (smaller cases with the same recipe).
    """
    if i == 0:
        n, m, r = overrides.get("n", 500), overrides.get("m", 400), overrides.get("r", 10)
        dens = overrides.get("density", 0.02)
        ptr, idx, val, Ws, Fs, c = planted(n, m, r, dens, seed, tag=0)
        return _problem(n, m, r, ptr, idx, val, seed, 0,
                        {"name": CONFIG_NAMES[0], "sweeps": 10, "c": c, "density": dens})
    if i in (1, 2):
        if i == 1:
            n, m, r, med, sweeps = 50_000, 100_000, 50, 80.0, 20
        else:
            n, m, r, med, sweeps = 100_000, 2_000_000, 100, 150.0 / math.exp(0.5), 10
        n = overrides.get("n", n)
        m = overrides.get("m", m)
        r = overrides.get("r", r)
        ptr, idx, val = corpus(n, m, med, 1.0, 2000, 1.1, 0.6, seed, tag=i,
                               workers=overrides.get("workers", 1), progress=overrides.get("progress"))
        if overrides.get("progress"):
            overrides["progress"]("CSR copy")
        return _problem(n, m, r, ptr, idx, val, seed, i,
                        {"name": CONFIG_NAMES[i] if (n, m) == ((50_000, 100_000) if i == 1 else (100_000, 2_000_000)) else f"corpus {n}x{m} r={r}",
                         "sweeps": sweeps})
    raise ValueError(f"config {i}: use batched_configs() / serving_* for 3 and 4")


def _batched_member(args):
    n, m, r, dens, seed, p = args
    ptr, idx, val, Ws, Fs, c = planted(n, m, r, dens, seed, tag=1000 + p)
    return _problem(n, m, r, ptr, idx, val, seed, 1000 + p,
                    {"name": f"batched[{p}]", "sweeps": 10, "density": dens})


def batched_configs(seed: int = 0, count: int = 64, scale: float = 1.0, workers: int = 1):
    """64 independent planted problems: n ~ U{1k..20k}, m ~ U{1k..50k}, r ~ U{10,16,32,64},
    density ~ U[0.1%, 2%], planted rank = r.  ``scale`` < 1 shrinks n and m (tests).
    ``workers`` > 1 generates the members in forked worker processes (same result; call
    it before the process uses a GPU)."""
    g = _rng(0xBA7C, seed)
    specs = []
    for p in range(count):
        n = max(8, int(g.integers(1000, 20001) * scale))
        m = max(8, int(g.integers(1000, 50001) * scale))
        r = int(g.choice([10, 16, 32, 64]))
        dens = float(g.uniform(0.001, 0.02))
        specs.append((n, m, r, dens, seed, p))
    if workers <= 1:
        return [_batched_member(s) for s in specs]
    import concurrent.futures as cf
    import multiprocessing as mp
    # largest members first, so that the pool's tail is short
    order = sorted(range(count), key=lambda p: -specs[p][0] * specs[p][1] * specs[p][3])
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        done = dict(zip(order, ex.map(_batched_member, [specs[p] for p in order])))
    return [done[p] for p in range(count)]


def serving_model(n: int = 50_000, r: int = 100, seed: int = 0) -> np.ndarray:
    """Resident model for fold-in serving: W (n x r, point-major) iid Gamma(0.1, 1)."""
    g = _rng(0x5E7E, seed)
    return g.gamma(0.1, 1.0, size=(n, r)).astype(np.float32)


def serving_requests(count: int, n: int = 50_000, rate: float = 20_000.0, seed: int = 0,
                     median_len: float = 80.0, max_len: int = 5000):
    """Poisson-arriving single documents: arrival times (s), CSC-style (ptr, idx, val).

    Lengths LogNormal(ln 80, 1) clipped to [1, 5000]; Zipf(1.1) word ids with the same
    relabelling recipe as ``corpus``; counts 1 + Geometric_0(0.6)."""
    g = _rng(0x5E7F, seed)
    arrivals = np.cumsum(g.exponential(1.0 / rate, count))
    ptr, idx, val = corpus(n, count, median_len, 1.0, max_len, 1.1, 0.6, seed, tag=4)
    return arrivals, ptr, idx, val
