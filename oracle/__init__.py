"""ctypes wrapper of the FP64 CPU oracle (``nmfkl_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and by the
benchmark's CPU-baseline leg.  The product library never loads it, and it imports nothing
from the product package.

Every array handed to the oracle is converted to float64 / int32 / int64 C-contiguous
copies here; results come back as float64 numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nmfkl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")


class Params(ctypes.Structure):
    _fields_ = [
        ("alpha_W", ctypes.c_double), ("alpha_F", ctypes.c_double),
        ("beta_W", ctypes.c_double), ("beta_F", ctypes.c_double),
        ("eps_log", ctypes.c_double), ("eps_g", ctypes.c_double), ("eps_x", ctypes.c_double),
        ("t_max", ctypes.c_int32), ("j_max", ctypes.c_int32),
        ("literal_break", ctypes.c_int32), ("guard", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("foldin_max_passes", ctypes.c_int32), ("foldin_tol", ctypes.c_double),
    ]


class Stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in
                ("coords", "evals", "steps", "halvings", "rejects", "tmax_hits")]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


def params(**kw) -> Params:
    """Defaults: alpha = beta = 0, eps_log 1e-10, eps_g 1e-5, eps_x 0.1 (Section 3),
    t_max 16, j_max 8, magnitude break, guard on, seed 0, fold-in 200 passes / tol 1e-5."""
    p = Params(alpha_W=0.0, alpha_F=0.0, beta_W=0.0, beta_F=0.0, eps_log=1e-10, eps_g=1e-5,
               eps_x=0.1, t_max=16, j_max=8, literal_break=0, guard=1, seed=0,
               foldin_max_passes=200, foldin_tol=1e-5)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def build(force: bool = False, src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


_lib = None


def load(path: str | None = None):
    """Load (building if needed) the oracle library; a custom path loads a separate copy."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    lib = ctypes.CDLL(path or build())
    lib.orc_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
    lib.orc_permutation.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.c_int32, _i32p]
    lib.orc_factor_sums.argtypes = [ctypes.c_int64, ctypes.c_int32, _f64p, _f64p]
    lib.orc_coordinate_derivatives.argtypes = [
        ctypes.c_int64, _i32p, _f64p, _f64p, ctypes.c_int32, ctypes.c_int32, _f64p,
        ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
        ctypes.POINTER(ctypes.c_double)]
    lib.orc_subproblem_value.argtypes = [ctypes.c_int64, _i32p, _f64p, _f64p, ctypes.c_int32,
                                         _f64p, _f64p, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double]
    lib.orc_subproblem_value.restype = ctypes.c_double
    lib.orc_coordinate_update.argtypes = [
        ctypes.c_int64, _i32p, _f64p, _f64p, ctypes.c_int32, _f64p, _f64p, ctypes.c_double,
        ctypes.c_double, ctypes.c_int32, ctypes.POINTER(Params), _f64p, _f64p,
        ctypes.POINTER(Stats)]
    lib.orc_alg2.argtypes = [ctypes.c_int64, _i32p, _f64p, _f64p, ctypes.c_int32, _f64p, _f64p,
                             ctypes.c_double, ctypes.c_double, _i32p, ctypes.POINTER(Params),
                             _f64p, _f64p, ctypes.POINTER(Stats)]
    for name in ("orc_sweep_F", "orc_sweep_W"):
        getattr(lib, name).argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _i64p,
                                       _i32p, _f64p, _f64p, _f64p, _i32p,
                                       ctypes.POINTER(Params), ctypes.POINTER(Stats), _f64p]
    lib.orc_objective.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _i64p, _i32p,
                                  _f64p, _f64p, _f64p]
    lib.orc_objective.restype = ctypes.c_double
    lib.orc_column_kl.argtypes = [ctypes.c_int64, _i32p, _f64p, _f64p, ctypes.c_int32, _f64p,
                                  _f64p]
    lib.orc_column_kl.restype = ctypes.c_double
    lib.orc_foldin.argtypes = [ctypes.c_int32, ctypes.c_int32, _f64p, ctypes.c_int64, _i64p,
                               _i32p, _f64p, ctypes.POINTER(Params), _f64p, _i32p, _f64p,
                               ctypes.POINTER(Stats)]
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    if path is None:
        _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def philox(ctr, key, lib=None) -> np.ndarray:
    out = np.zeros(4, np.uint64)
    (lib or load()).orc_philox4x64_10(np.asarray(ctr, np.uint64), np.asarray(key, np.uint64), out)
    return out


def permutation(seed: int, t: int, stream: int, r: int, lib=None) -> np.ndarray:
    ids = np.zeros(r, np.int32)
    (lib or load()).orc_permutation(seed, t, stream, r, ids)
    return ids


def factor_sums(A, lib=None) -> np.ndarray:
    A = _f64(A)
    out = np.zeros(A.shape[1], np.float64)
    (lib or load()).orc_factor_sums(A.shape[0], A.shape[1], A, out)
    return out


def coordinate_derivatives(idx, v, A, k, Ax, sumA_k, xk, alpha=0.0, beta=0.0, eps_log=1e-10,
                           lib=None):
    g, h, P = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    A = _f64(A)
    (lib or load()).orc_coordinate_derivatives(len(idx), _i32(idx), _f64(v), A, A.shape[1], k,
                                               _f64(Ax), sumA_k, xk, alpha, beta, eps_log,
                                               ctypes.byref(g), ctypes.byref(h), ctypes.byref(P))
    return g.value, h.value, P.value


def subproblem_value(idx, v, A, sumA, x, alpha=0.0, beta=0.0, eps_log=1e-10, lib=None) -> float:
    A = _f64(A)
    return (lib or load()).orc_subproblem_value(len(idx), _i32(idx), _f64(v), A, A.shape[1],
                                                _f64(sumA), _f64(x), alpha, beta, eps_log)


def model_at(idx, A, x):
    """Plain [Ax] at the listed points (numpy matmul)."""
    return _f64(A)[_i32(idx)] @ _f64(x)


def coordinate_update(idx, v, A, sumA, x, k, prm=None, alpha=0.0, beta=0.0, Ax=None, lib=None):
    """One coordinate's inner loop; returns (x_new, Ax_new, stats)."""
    A = _f64(A)
    x = _f64(x).copy()
    Ax = model_at(idx, A, x) if Ax is None else _f64(Ax).copy()
    Axn = np.zeros_like(Ax)
    st = Stats()
    prm = prm or params()
    (lib or load()).orc_coordinate_update(len(idx), _i32(idx), _f64(v), A, A.shape[1],
                                          _f64(sumA), x, alpha, beta, k, ctypes.byref(prm), Ax,
                                          Axn, ctypes.byref(st))
    return x, Ax, st.as_dict()


def alg2(idx, v, A, sumA, x, ids, prm=None, alpha=0.0, beta=0.0, lib=None):
    """Alg. 2 on one column; returns (x_new, Ax_new, stats)."""
    A = _f64(A)
    x = _f64(x).copy()
    L = len(idx)
    Ax = np.zeros(max(L, 1))
    Axn = np.zeros(max(L, 1))
    st = Stats()
    prm = prm or params()
    (lib or load()).orc_alg2(L, _i32(idx), _f64(v), A, A.shape[1], _f64(sumA), x, alpha, beta,
                             _i32(ids), ctypes.byref(prm), Ax, Axn, ctypes.byref(st))
    return x, Ax[:L], st.as_dict()


def sweep_F(prob, W, F, ids, prm=None, lib=None):
    """F-half of Alg. 1; returns (F_new, sumW, stats)."""
    F = _f64(F).copy()
    sw = np.zeros(prob.r, np.float64)
    st = Stats()
    (lib or load()).orc_sweep_F(prob.n, prob.m, prob.r, _i64(prob.csc_ptr), _i32(prob.csc_idx),
                                _f64(prob.csc_val), _f64(W), F, _i32(ids),
                                ctypes.byref(prm or params()), ctypes.byref(st), sw)
    return F, sw, st.as_dict()


def sweep_W(prob, F, W, ids, prm=None, lib=None):
    """W-half of Alg. 1; returns (W_new, sumF, stats)."""
    W = _f64(W).copy()
    sf = np.zeros(prob.r, np.float64)
    st = Stats()
    (lib or load()).orc_sweep_W(prob.n, prob.m, prob.r, _i64(prob.csr_ptr), _i32(prob.csr_idx),
                                _f64(prob.csr_val), _f64(F), W, _i32(ids),
                                ctypes.byref(prm or params()), ctypes.byref(st), sf)
    return W, sf, st.as_dict()


def objective(prob, W, F, lib=None) -> float:
    return (lib or load()).orc_objective(prob.n, prob.m, prob.r, _i64(prob.csc_ptr),
                                         _i32(prob.csc_idx), _f64(prob.csc_val), _f64(W), _f64(F))


def column_kl(idx, v, A, sumA, x, lib=None) -> float:
    A = _f64(A)
    return (lib or load()).orc_column_kl(len(idx), _i32(idx), _f64(v), A, A.shape[1], _f64(sumA),
                                         _f64(x))


def foldin(W, doc_ptr, word_idx, counts, prm=None, lib=None):
    """Fold-in of documents with W fixed; returns (F (ndocs x r), passes, kl, stats)."""
    W = _f64(W)
    nd = len(doc_ptr) - 1
    F = np.zeros((nd, W.shape[1]), np.float64)
    passes = np.zeros(nd, np.int32)
    kl = np.zeros(nd, np.float64)
    st = Stats()
    (lib or load()).orc_foldin(W.shape[0], W.shape[1], W, nd, _i64(doc_ptr), _i32(word_idx),
                               _f64(counts), ctypes.byref(prm or params()), F, passes, kl,
                               ctypes.byref(st))
    return F, passes, kl, st.as_dict()


def run(prob, sweeps: int, prm=None, seed: int = 0, W=None, F=None, t0: int = 0, lib=None):
    """Alg. 1 for a fixed number of outer iterations (sweeps) from (W0, F0).

    Returns (W, F, D) with D[t] the eq. 1 objective after sweep t."""
    prm = prm or params(seed=seed)
    W = _f64(prob.W0 if W is None else W).copy()
    F = _f64(prob.F0 if F is None else F).copy()
    D = []
    for t in range(t0, t0 + sweeps):
        ids = permutation(prm.seed, t, 0, prob.r, lib)
        F, _, _ = sweep_F(prob, W, F, ids, prm, lib)
        W, _, _ = sweep_W(prob, F, W, ids, prm, lib)
        D.append(objective(prob, W, F, lib))
    return W, F, np.array(D)


def set_threads(t: int, lib=None):
    (lib or load()).orc_set_num_threads(int(t))


def threads(lib=None) -> int:
    return int((lib or load()).orc_num_threads())
