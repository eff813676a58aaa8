"""MI355X NMF-KL randomized coordinate descent: Python binding of ``libnmfkl.so``.

The binding only marshals arguments: torch tensors give device pointers and the HIP
stream, and every step of the method runs in the library's kernels.  The names mirror the
C ABI declared in ``include/nmfkl.h``.  There is no fallback: if the library is not built
or cannot be loaded, every call raises.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

import numpy as np

from .build import LIB as _LIB_PATH

__all__ = [
    "NmfklError", "NmfklParams", "NmfklProblem", "NmfklStats", "load", "nmfkl_params_default",
    "nmfkl_permutation", "nmfkl_create", "nmfkl_sweep_F", "nmfkl_sweep_W", "nmfkl_objective",
    "nmfkl_invalidate_model", "nmfkl_get_stats", "nmfkl_get_timings", "nmfkl_reset_timings",
    "nmfkl_destroy", "nmfkl_last_error", "DeviceProblem", "upload", "upload_host_v", "Handle", "EXPORTED_SYMBOLS",
]

NMFKL_OK = 0
ERRORS = {-1: "NMFKL_E_INVAL", -2: "NMFKL_E_NOMEM", -3: "NMFKL_E_DEVICE", -4: "NMFKL_E_NONFINITE",
          -5: "NMFKL_E_BUSY", -6: "NMFKL_E_UNSUPPORTED"}
R_MAX = 128

EXPORTED_SYMBOLS = [
    "nmfkl_params_default", "nmfkl_permutation", "nmfkl_create", "nmfkl_sweep_F", "nmfkl_sweep_W",
    "nmfkl_objective", "nmfkl_objective_carried", "nmfkl_objective_enqueue", "nmfkl_objective_read",
    "nmfkl_invalidate_model", "nmfkl_get_stats", "nmfkl_get_timings",
    "nmfkl_reset_timings", "nmfkl_destroy", "nmfkl_last_error",
    "nmfkl_model_create", "nmfkl_foldin", "nmfkl_foldin_noalloc", "nmfkl_model_get_stats", "nmfkl_model_last_error",
    "nmfkl_model_destroy", "nmfkl_server_create", "nmfkl_server_submit", "nmfkl_server_poll",
    "nmfkl_server_pending", "nmfkl_server_last_error", "nmfkl_server_destroy", "nmfkl_server_cancel",
    "nmfkl_server_now",
    "nmfkl_batch_create", "nmfkl_batch_run", "nmfkl_batch_objective", "nmfkl_batch_tune",
    "nmfkl_batch_get_info", "nmfkl_batch_last_error", "nmfkl_batch_destroy",
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
        ("bin_shift", ctypes.c_int32), ("tile_bf16", ctypes.c_int32),
        ("out_of_core", ctypes.c_int32), ("ooc_chunk_nnz", ctypes.c_int64),
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
                ("coords", "evals", "steps", "halvings", "rejects", "tmax_hits", "zeros_W", "zeros_F")]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


TIMED = ["sums_F", "fused_F", "long_F", "sums_W", "fused_W", "long_W", "model", "terms"]


class NmfklKernelTiming(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_double), ("launches", ctypes.c_int64),
                ("gather_bytes", ctypes.c_double), ("updates", ctypes.c_double)]


class NmfklTimings(ctypes.Structure):
    _fields_ = [("k", NmfklKernelTiming * len(TIMED))]

    def as_dict(self):
        return {name: {f: getattr(self.k[i], f) for f, _ in NmfklKernelTiming._fields_}
                for i, name in enumerate(TIMED)}


class NmfklBatchInfo(ctypes.Structure):
    _fields_ = [("nprob", ctypes.c_int32), ("bin_shift", ctypes.c_int32), ("tuning", ctypes.c_int32),
                ("graph_cooperative", ctypes.c_int32), ("fused_blocks", ctypes.c_int32 * 2),
                ("long_parts", ctypes.c_int32 * 2), ("long_rounds", ctypes.c_int32 * 2),
                ("nnz_total", ctypes.c_int64)]

    def as_dict(self):
        out = {}
        for f, _ in self._fields_:
            v = getattr(self, f)
            out[f] = list(v) if isinstance(v, ctypes.Array) else int(v)
        return out


class NmfklResult(ctypes.Structure):
    _fields_ = [("req_id", ctypes.c_uint64), ("passes", ctypes.c_int32), ("status", ctypes.c_int32),
                ("kl", ctypes.c_double), ("t_submit", ctypes.c_double), ("t_done", ctypes.c_double)]


RESULT_EXPIRED = 1
RESULT_CANCELLED = 2


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
    lib.nmfkl_objective_enqueue.argtypes = [vp]
    lib.nmfkl_objective_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.nmfkl_invalidate_model.argtypes = [vp]
    lib.nmfkl_get_stats.argtypes = [vp, ctypes.POINTER(NmfklStats)]
    lib.nmfkl_get_timings.argtypes = [vp, ctypes.POINTER(NmfklTimings)]
    lib.nmfkl_reset_timings.argtypes = [vp]
    lib.nmfkl_destroy.argtypes = [vp]
    lib.nmfkl_last_error.argtypes = [vp]
    lib.nmfkl_last_error.restype = ctypes.c_char_p
    lib.nmfkl_model_create.argtypes = [vp, i32, i32, ctypes.POINTER(NmfklParams), vp, ctypes.POINTER(vp)]
    lib.nmfkl_foldin.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    lib.nmfkl_foldin_noalloc.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    lib.nmfkl_model_get_stats.argtypes = [vp, ctypes.POINTER(NmfklStats)]
    lib.nmfkl_model_destroy.argtypes = [vp]
    lib.nmfkl_server_create.argtypes = [vp, i64, i32, i32, i32, ctypes.POINTER(vp)]
    lib.nmfkl_server_submit.argtypes = [vp, u64, i32, vp, vp, ctypes.c_double]
    lib.nmfkl_server_cancel.argtypes = [vp, u64]
    lib.nmfkl_server_now.argtypes = [ctypes.POINTER(ctypes.c_double)]
    lib.nmfkl_server_poll.argtypes = [vp, i32, ctypes.POINTER(NmfklResult), vp, ctypes.POINTER(ctypes.c_int32)]
    lib.nmfkl_server_pending.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.nmfkl_server_destroy.argtypes = [vp]
    lib.nmfkl_batch_create.argtypes = [i32, ctypes.POINTER(NmfklProblem), ctypes.POINTER(NmfklParams), vp,
                                       ctypes.POINTER(vp)]
    lib.nmfkl_batch_run.argtypes = [vp, i32, i32]
    lib.nmfkl_batch_objective.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.nmfkl_batch_tune.argtypes = [vp, i32, ctypes.POINTER(NmfklParams)]
    lib.nmfkl_batch_get_info.argtypes = [vp, ctypes.POINTER(NmfklBatchInfo)]
    lib.nmfkl_batch_destroy.argtypes = [vp]
    for name in ("nmfkl_model_last_error", "nmfkl_server_last_error", "nmfkl_batch_last_error"):
        getattr(lib, name).argtypes = [vp]
        getattr(lib, name).restype = ctypes.c_char_p
    for name in EXPORTED_SYMBOLS:
        if not name.endswith("last_error"):
            getattr(lib, name).restype = ctypes.c_int
    if path is None:
        if _lib is None:
            # atexit runs hooks last-in first-out: registered after torch's import, this one
            # runs before torch's own exit hooks
            atexit.register(_destroy_live_objects)
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

    def __init__(self, n, m, r, csc_ptr, csc_idx, csc_val, csr_ptr, csr_idx, csr_val, W, F, host_v=False):
        self.n, self.m, self.r = int(n), int(m), int(r)
        self.csc_ptr, self.csc_idx, self.csc_val = csc_ptr, csc_idx, csc_val
        self.csr_ptr, self.csr_idx, self.csr_val = csr_ptr, csr_idx, csr_val
        self.W, self.F = W, F
        self.host_v = host_v
        import torch
        for k, (t, dt) in enumerate(((csc_ptr, torch.int64), (csc_idx, torch.int32), (csc_val, torch.float32),
                                     (csr_ptr, torch.int64), (csr_idx, torch.int32), (csr_val, torch.float32),
                                     (W, torch.float32), (F, torch.float32))):
            on_device = not (host_v and k < 6)
            if t.dtype != dt or t.is_cuda != on_device or not t.is_contiguous():
                where = "device" if on_device else "host"
                raise ValueError(f"expected a contiguous {dt} {where} tensor, got {t.dtype} on {t.device}")
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


def upload_host_v(prob, device="cuda", W=None, F=None) -> DeviceProblem:
    """V's six arrays in pinned host memory (for params.out_of_core = 1), the factors on the
    device."""
    import torch
    h = lambda a: torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    return DeviceProblem(prob.n, prob.m, prob.r, h(prob.csc_ptr), h(prob.csc_idx), h(prob.csc_val),
                         h(prob.csr_ptr), h(prob.csr_idx), h(prob.csr_val),
                         d(np.asarray(prob.W0 if W is None else W, np.float32)),
                         d(np.asarray(prob.F0 if F is None else F, np.float32)), host_v=True)


# Every live native object (handle, model, server, batch), so that they can be destroyed at
# interpreter exit before torch and the HIP runtime tear down.  A destroy call during the
# interpreter's own finalisation (from __del__ of an object that outlived the exit hook, or of
# module globals) could reach HIP after its teardown began; __del__ therefore does nothing once
# the interpreter is finalising, and the exit hook below has already released what was live.
_live: "weakref.WeakSet[_Native]" = weakref.WeakSet()
_EXIT_ORDER = {"nmfkl_server_destroy": 0, "nmfkl_batch_destroy": 1, "nmfkl_destroy": 2,
               "nmfkl_model_destroy": 3}


class _Native:
    _destroy_fn = ""

    def _register(self):
        _live.add(self)

    def _release(self):
        if self._ptr:
            ptr, self._ptr = self._ptr, None
            return getattr(load(), self._destroy_fn)(ptr)
        return NMFKL_OK

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self._release()
        except Exception:
            pass


def _destroy_live_objects():
    """Exit hook: synchronise the device, then destroy the live objects (servers before the
    models they use)."""
    objs = sorted(list(_live), key=lambda o: _EXIT_ORDER.get(o._destroy_fn, 9))
    if not objs:
        return
    try:
        import torch
        if torch.cuda.is_initialized():
            torch.cuda.synchronize()
    except Exception:
        pass
    for o in objs:
        try:
            o._release()
        except Exception:
            pass


class Handle(_Native):
    """An nmfkl_handle plus references that keep its device tensors alive."""
    _destroy_fn = "nmfkl_destroy"

    def __init__(self, ptr: int, dev: DeviceProblem, stream):
        self._ptr = ptr
        self.dev = dev
        self.stream = stream
        self._register()


def nmfkl_create(dev: DeviceProblem, params: NmfklParams | None = None, stream=None) -> Handle:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    out = ctypes.c_void_p()
    prob = dev.struct()
    prm = params if params is not None else nmfkl_params_default()
    if bool(prm.out_of_core) != bool(getattr(dev, "host_v", False)):
        raise ValueError("params.out_of_core = 1 takes V in host memory (upload_host_v); 0 takes it on the device")
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


def nmfkl_objective_enqueue(h: Handle):
    _check(load().nmfkl_objective_enqueue(h._ptr), h._ptr)


def nmfkl_objective_read(h: Handle) -> float:
    d = ctypes.c_double()
    _check(load().nmfkl_objective_read(h._ptr, ctypes.byref(d)), h._ptr)
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


# ------------------------------------------------------------------ fold-in and serving
def _mcheck(rc, m=None):
    if rc != NMFKL_OK:
        msg = load().nmfkl_model_last_error(m)
        raise NmfklError(rc, msg.decode() if msg else "")


class Model(_Native):
    """An nmfkl_model over a resident W (device tensor n x r, kept alive here)."""
    _destroy_fn = "nmfkl_model_destroy"

    def __init__(self, ptr, W, r, stream):
        self._ptr, self.W, self.r, self.stream = ptr, W, r, stream
        self._register()


def nmfkl_model_create(W, params: NmfklParams | None = None, stream=None) -> Model:
    import torch
    if W.dtype != torch.float32 or not W.is_cuda or not W.is_contiguous() or W.dim() != 2:
        raise ValueError("W must be a contiguous float32 device tensor n x r")
    if stream is None:
        stream = torch.cuda.current_stream()
    out = ctypes.c_void_p()
    prm = params if params is not None else nmfkl_params_default()
    _mcheck(load().nmfkl_model_create(W.data_ptr(), W.shape[0], W.shape[1], ctypes.byref(prm),
                                      _stream_ptr(stream), ctypes.byref(out)))
    return Model(out.value, W, W.shape[1], stream)


def nmfkl_foldin(m: Model, doc_ptr, word_idx, counts):
    """Fold in documents (device tensors, CSC form); returns device tensors (F, passes, kl)."""
    import torch
    nd = doc_ptr.numel() - 1
    dev = doc_ptr.device
    F = torch.empty((nd, m.r), dtype=torch.float32, device=dev)
    passes = torch.empty(nd, dtype=torch.int32, device=dev)
    kl = torch.empty(nd, dtype=torch.float64, device=dev)
    _mcheck(load().nmfkl_foldin(m._ptr, nd, doc_ptr.data_ptr(), word_idx.data_ptr(), counts.data_ptr(),
                                F.data_ptr(), passes.data_ptr(), kl.data_ptr()), m._ptr)
    return F, passes, kl


def nmfkl_foldin_noalloc(m: Model, doc_ptr, word_idx, counts, F, passes, kl):
    """nmfkl_foldin into caller-provided device outputs (F ndocs x r float32, passes int32,
    kl float64); the library allocates nothing (at most 16384 documents per call)."""
    import torch
    nd = doc_ptr.numel() - 1
    for t, dt, shape in ((F, torch.float32, (nd, m.r)), (passes, torch.int32, (nd,)), (kl, torch.float64, (nd,))):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shape:
            raise ValueError(f"output must be a contiguous {dt} device tensor of shape {shape}")
    for t, dt in ((doc_ptr, torch.int64), (word_idx, torch.int32), (counts, torch.float32)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"documents must be contiguous device tensors ({dt})")
    _mcheck(load().nmfkl_foldin_noalloc(m._ptr, nd, doc_ptr.data_ptr(), word_idx.data_ptr(), counts.data_ptr(),
                                        F.data_ptr(), passes.data_ptr(), kl.data_ptr()), m._ptr)
    return F, passes, kl


def nmfkl_model_get_stats(m: Model) -> dict:
    s = NmfklStats()
    _mcheck(load().nmfkl_model_get_stats(m._ptr, ctypes.byref(s)), m._ptr)
    return s.as_dict()


def nmfkl_model_destroy(m: Model):
    if m._ptr:
        rc = load().nmfkl_model_destroy(m._ptr)
        m._ptr = None
        _mcheck(rc)


def _scheck(rc, s=None):
    if rc != NMFKL_OK:
        msg = load().nmfkl_server_last_error(s)
        raise NmfklError(rc, msg.decode() if msg else "")


class Server(_Native):
    """An nmfkl_server over a model (kept alive here)."""
    _destroy_fn = "nmfkl_server_destroy"

    def __init__(self, ptr, model):
        self._ptr, self.model = ptr, model
        self._register()


def nmfkl_server_create(m: Model, mem_budget_bytes: int, lanes: int = 8, lane_docs: int = 256,
                        max_queued: int = 0) -> Server:
    out = ctypes.c_void_p()
    _scheck(load().nmfkl_server_create(m._ptr, int(mem_budget_bytes), int(lanes), int(lane_docs), int(max_queued),
                                       ctypes.byref(out)))
    return Server(out.value, m)


def nmfkl_server_submit(s: Server, req_id: int, word_idx: np.ndarray, counts: np.ndarray,
                        timeout_s: float = 0.0) -> int:
    """Returns NMFKL_OK, or an admission code when the document cannot wait now: NMFKL_E_NOMEM
    (the memory budget is full) or NMFKL_E_BUSY (every waiting slot is taken).  Raises on
    malformed or unsupported documents."""
    idx = np.ascontiguousarray(word_idx, dtype=np.int32)
    val = np.ascontiguousarray(counts, dtype=np.float32)
    rc = load().nmfkl_server_submit(s._ptr, int(req_id), int(idx.size), idx.ctypes.data, val.ctypes.data,
                                    float(timeout_s))
    if rc not in (NMFKL_OK, -2, -5):
        _scheck(rc, s._ptr)
    return rc


def nmfkl_server_cancel(s: Server, req_id: int) -> int:
    """Withdraws a waiting document (returned later with status RESULT_CANCELLED); returns
    NMFKL_OK, or NMFKL_E_INVAL when no waiting document has this id."""
    return load().nmfkl_server_cancel(s._ptr, int(req_id))


def nmfkl_server_now() -> float:
    t = ctypes.c_double()
    _scheck(load().nmfkl_server_now(ctypes.byref(t)))
    return t.value


def nmfkl_server_poll(s: Server, max_results: int = 4096):
    """Finished documents: list of (req_id, passes, kl, t_submit, t_done, f, status)."""
    r = s.model.r
    res = (NmfklResult * max(max_results, 1))()
    f = np.empty((max(max_results, 1), r), dtype=np.float32)
    n = ctypes.c_int32()
    _scheck(load().nmfkl_server_poll(s._ptr, max_results, res, f.ctypes.data, ctypes.byref(n)), s._ptr)
    return [(res[k].req_id, res[k].passes, res[k].kl, res[k].t_submit, res[k].t_done, f[k].copy(), res[k].status)
            for k in range(n.value)]


class PollBuffer:
    """Reusable result buffers for nmfkl_server_poll_into (no allocation per poll)."""

    def __init__(self, max_results: int, r: int):
        self.max_results = max_results
        self.res = (NmfklResult * max_results)()
        self.f = np.empty((max_results, r), dtype=np.float32)
        self.n = ctypes.c_int32()


def nmfkl_server_poll_into(s: Server, buf: PollBuffer) -> int:
    """Like nmfkl_server_poll into buf.res / buf.f; returns the number of results."""
    _scheck(load().nmfkl_server_poll(s._ptr, buf.max_results, buf.res, buf.f.ctypes.data,
                                     ctypes.byref(buf.n)), s._ptr)
    return buf.n.value


def nmfkl_server_pending(s: Server):
    q, w = ctypes.c_int64(), ctypes.c_int64()
    _scheck(load().nmfkl_server_pending(s._ptr, ctypes.byref(q), ctypes.byref(w)), s._ptr)
    return q.value, w.value


def nmfkl_server_destroy(s: Server):
    if s._ptr:
        rc = load().nmfkl_server_destroy(s._ptr)
        s._ptr = None
        _scheck(rc)


# ------------------------------------------------------------------ batched problems
def _bcheck(rc, b=None):
    if rc != NMFKL_OK:
        msg = load().nmfkl_batch_last_error(b)
        raise NmfklError(rc, msg.decode() if msg else "")


class Batch(_Native):
    """An nmfkl_batch over device problems (kept alive here)."""
    _destroy_fn = "nmfkl_batch_destroy"

    def __init__(self, ptr, devs, stream):
        self._ptr, self.devs, self.stream = ptr, devs, stream
        self._register()


def nmfkl_batch_create(devs, params: NmfklParams | None = None, stream=None) -> Batch:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    arr = (NmfklProblem * len(devs))(*[d.struct() for d in devs])
    out = ctypes.c_void_p()
    prm = params if params is not None else nmfkl_params_default()
    _bcheck(load().nmfkl_batch_create(len(devs), arr, ctypes.byref(prm), _stream_ptr(stream), ctypes.byref(out)))
    return Batch(out.value, list(devs), stream)


def nmfkl_batch_run(b: Batch, t0: int, nsweeps: int):
    _bcheck(load().nmfkl_batch_run(b._ptr, int(t0), int(nsweeps)), b._ptr)


def nmfkl_batch_objective(b: Batch) -> np.ndarray:
    D = np.empty(len(b.devs), dtype=np.float64)
    _bcheck(load().nmfkl_batch_objective(b._ptr, D.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), b._ptr)
    return D


def nmfkl_batch_tune(b: Batch, t: int = 0) -> NmfklParams:
    out = NmfklParams()
    _bcheck(load().nmfkl_batch_tune(b._ptr, int(t), ctypes.byref(out)), b._ptr)
    return out


def nmfkl_batch_get_info(b: Batch) -> dict:
    info = NmfklBatchInfo()
    _bcheck(load().nmfkl_batch_get_info(b._ptr, ctypes.byref(info)), b._ptr)
    return info.as_dict()


def nmfkl_batch_destroy(b: Batch):
    if b._ptr:
        rc = load().nmfkl_batch_destroy(b._ptr)
        b._ptr = None
        _bcheck(rc)
