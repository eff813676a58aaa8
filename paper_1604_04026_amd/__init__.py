"""MI355X NMF-KL randomized coordinate descent: Python binding of ``libnmfkl.so``.

The binding only marshals arguments: torch tensors give device pointers and the HIP
stream, and every step of the method runs in the library's kernels.  The names mirror the
C ABI declared in ``include/nmfkl.h``.  There is no fallback: if the library is not built
or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB as _LIB_PATH

__all__ = [
    "NmfklError", "NmfklParams", "NmfklProblem", "NmfklStats", "load", "nmfkl_params_default",
    "nmfkl_permutation", "nmfkl_create", "nmfkl_sweep_F", "nmfkl_sweep_W", "nmfkl_objective",
    "nmfkl_invalidate_model", "nmfkl_get_stats", "nmfkl_get_timings", "nmfkl_reset_timings",
    "nmfkl_destroy", "nmfkl_last_error", "DeviceProblem", "upload", "Handle", "EXPORTED_SYMBOLS",
]

NMFKL_OK = 0
ERRORS = {-1: "NMFKL_E_INVAL", -2: "NMFKL_E_NOMEM", -3: "NMFKL_E_DEVICE", -4: "NMFKL_E_NONFINITE",
          -5: "NMFKL_E_BUSY", -6: "NMFKL_E_UNSUPPORTED"}
R_MAX = 128

EXPORTED_SYMBOLS = [
    "nmfkl_params_default", "nmfkl_permutation", "nmfkl_create", "nmfkl_sweep_F", "nmfkl_sweep_W",
    "nmfkl_objective", "nmfkl_objective_carried", "nmfkl_invalidate_model", "nmfkl_get_stats", "nmfkl_get_timings",
    "nmfkl_reset_timings", "nmfkl_destroy", "nmfkl_last_error",
]


class NmfklError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{ERRORS.get(code, code)}: {message}")
        self.code = code
        self.message = message


class NmfklParams(ctypes.Structure):
    _fields_ = [
        ("alpha_W", ctypes.c_double), ("alpha_F", ctypes.c_double),
        ("beta_W", ctypes.c_double), ("beta_F", ctypes.c_double),
        ("eps_log", ctypes.c_double), ("eps_g", ctypes.c_double), ("eps_x", ctypes.c_double),
        ("t_max", ctypes.c_int32), ("j_max", ctypes.c_int32),
        ("literal_break", ctypes.c_int32), ("guard", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("foldin_max_passes", ctypes.c_int32), ("foldin_tol", ctypes.c_double),
        ("refresh_model", ctypes.c_int32), ("collect_stats", ctypes.c_int32),
        ("collect_timings", ctypes.c_int32), ("tuning", ctypes.c_int32),
    ]


class NmfklProblem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("m", ctypes.c_int32), ("r", ctypes.c_int32),
        ("nnz", ctypes.c_int64),
        ("csc_ptr", ctypes.c_void_p), ("csc_idx", ctypes.c_void_p), ("csc_val", ctypes.c_void_p),
        ("csr_ptr", ctypes.c_void_p), ("csr_idx", ctypes.c_void_p), ("csr_val", ctypes.c_void_p),
        ("W", ctypes.c_void_p), ("F", ctypes.c_void_p),
    ]


class NmfklStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in
                ("coords", "evals", "steps", "halvings", "rejects", "tmax_hits")]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


TIMED = ["sums_F", "fused_F", "long_F", "sums_W", "fused_W", "long_W", "model"]


class NmfklKernelTiming(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_double), ("launches", ctypes.c_int64),
                ("gather_bytes", ctypes.c_double), ("updates", ctypes.c_double)]


class NmfklTimings(ctypes.Structure):
    _fields_ = [("k", NmfklKernelTiming * len(TIMED))]

    def as_dict(self):
        return {name: {f: getattr(self.k[i], f) for f, _ in NmfklKernelTiming._fields_}
                for i, name in enumerate(TIMED)}


_lib = None


def load(path: str | None = None):
    """Load libnmfkl.so.  torch is imported first so that the library binds to the HIP
    runtime torch already loaded (same soname) and shares its device allocations."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    import torch  # noqa: F401  (HIP runtime first)
    p = path or _LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is not built: run __graft_entry__.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(p)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    lib.nmfkl_params_default.argtypes = [ctypes.POINTER(NmfklParams)]
    lib.nmfkl_permutation.argtypes = [u64, u64, u64, i32, ctypes.POINTER(ctypes.c_int32)]
    lib.nmfkl_create.argtypes = [ctypes.POINTER(NmfklProblem), ctypes.POINTER(NmfklParams), vp,
                                 ctypes.POINTER(vp)]
    lib.nmfkl_sweep_F.argtypes = [vp, i32]
    lib.nmfkl_sweep_W.argtypes = [vp, i32]
    lib.nmfkl_objective.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.nmfkl_objective_carried.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.nmfkl_invalidate_model.argtypes = [vp]
    lib.nmfkl_get_stats.argtypes = [vp, ctypes.POINTER(NmfklStats)]
    lib.nmfkl_get_timings.argtypes = [vp, ctypes.POINTER(NmfklTimings)]
    lib.nmfkl_reset_timings.argtypes = [vp]
    lib.nmfkl_destroy.argtypes = [vp]
    lib.nmfkl_last_error.argtypes = [vp]
    lib.nmfkl_last_error.restype = ctypes.c_char_p
    for name in EXPORTED_SYMBOLS:
        if name not in ("nmfkl_last_error",):
            getattr(lib, name).restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def _check(rc: int, h=None):
    if rc != NMFKL_OK:
        msg = load().nmfkl_last_error(h)
        raise NmfklError(rc, msg.decode() if msg else "")


def nmfkl_last_error(h=None) -> str:
    m = load().nmfkl_last_error(h._ptr if isinstance(h, Handle) else h)
    return m.decode() if m else ""


def nmfkl_params_default(**overrides) -> NmfklParams:
    p = NmfklParams()
    _check(load().nmfkl_params_default(ctypes.byref(p)))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def nmfkl_permutation(seed: int, t: int, stream: int, r: int) -> np.ndarray:
    ids = (ctypes.c_int32 * max(int(r), 1))()
    _check(load().nmfkl_permutation(seed, t, stream, r, ids))
    return np.frombuffer(ids, dtype=np.int32)[:r].copy()


def _stream_ptr(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class DeviceProblem:
    """Device copies (torch tensors) of V in CSC and CSR form and of the two factors."""

    def __init__(self, n, m, r, csc_ptr, csc_idx, csc_val, csr_ptr, csr_idx, csr_val, W, F):
        self.n, self.m, self.r = int(n), int(m), int(r)
        self.csc_ptr, self.csc_idx, self.csc_val = csc_ptr, csc_idx, csc_val
        self.csr_ptr, self.csr_idx, self.csr_val = csr_ptr, csr_idx, csr_val
        self.W, self.F = W, F
        import torch
        for t, dt in ((csc_ptr, torch.int64), (csc_idx, torch.int32), (csc_val, torch.float32),
                      (csr_ptr, torch.int64), (csr_idx, torch.int32), (csr_val, torch.float32),
                      (W, torch.float32), (F, torch.float32)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"expected a contiguous {dt} device tensor, got {t.dtype} on {t.device}")
        if tuple(W.shape) != (self.n, self.r) or tuple(F.shape) != (self.m, self.r):
            raise ValueError("W must be n x r and F m x r")

    @property
    def nnz(self) -> int:
        return int(self.csc_idx.numel())

    def struct(self) -> NmfklProblem:
        return NmfklProblem(self.n, self.m, self.r, self.nnz, self.csc_ptr.data_ptr(),
                            self.csc_idx.data_ptr(), self.csc_val.data_ptr(),
                            self.csr_ptr.data_ptr(), self.csr_idx.data_ptr(),
                            self.csr_val.data_ptr(), self.W.data_ptr(), self.F.data_ptr())


def upload(prob, device="cuda", W=None, F=None) -> DeviceProblem:
    """Copy a host problem (numpy arrays, see ``workloads``) to device tensors."""
    import torch
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    return DeviceProblem(prob.n, prob.m, prob.r, t(prob.csc_ptr), t(prob.csc_idx), t(prob.csc_val),
                         t(prob.csr_ptr), t(prob.csr_idx), t(prob.csr_val),
                         t(np.asarray(prob.W0 if W is None else W, np.float32)),
                         t(np.asarray(prob.F0 if F is None else F, np.float32)))


class Handle:
    """An nmfkl_handle plus references that keep its device tensors alive."""

    def __init__(self, ptr: int, dev: DeviceProblem, stream):
        self._ptr = ptr
        self.dev = dev
        self.stream = stream

    def __del__(self):
        try:
            if self._ptr:
                load().nmfkl_destroy(self._ptr)
                self._ptr = None
        except Exception:
            pass


def nmfkl_create(dev: DeviceProblem, params: NmfklParams | None = None, stream=None) -> Handle:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    out = ctypes.c_void_p()
    prob = dev.struct()
    prm = params if params is not None else nmfkl_params_default()
    _check(load().nmfkl_create(ctypes.byref(prob), ctypes.byref(prm), _stream_ptr(stream),
                               ctypes.byref(out)))
    return Handle(out.value, dev, stream)


def nmfkl_sweep_F(h: Handle, t: int):
    _check(load().nmfkl_sweep_F(h._ptr, int(t)), h._ptr)


def nmfkl_sweep_W(h: Handle, t: int):
    _check(load().nmfkl_sweep_W(h._ptr, int(t)), h._ptr)


def nmfkl_objective(h: Handle) -> float:
    d = ctypes.c_double()
    _check(load().nmfkl_objective(h._ptr, ctypes.byref(d)), h._ptr)
    return d.value


def nmfkl_objective_carried(h: Handle) -> float:
    d = ctypes.c_double()
    _check(load().nmfkl_objective_carried(h._ptr, ctypes.byref(d)), h._ptr)
    return d.value


def nmfkl_invalidate_model(h: Handle):
    _check(load().nmfkl_invalidate_model(h._ptr), h._ptr)


def nmfkl_get_stats(h: Handle) -> dict:
    s = NmfklStats()
    _check(load().nmfkl_get_stats(h._ptr, ctypes.byref(s)), h._ptr)
    return s.as_dict()


def nmfkl_get_timings(h: Handle) -> dict:
    t = NmfklTimings()
    _check(load().nmfkl_get_timings(h._ptr, ctypes.byref(t)), h._ptr)
    return t.as_dict()


def nmfkl_reset_timings(h: Handle):
    _check(load().nmfkl_reset_timings(h._ptr), h._ptr)


def nmfkl_destroy(h: Handle):
    if h._ptr:
        rc = load().nmfkl_destroy(h._ptr)
        h._ptr = None
        _check(rc)
