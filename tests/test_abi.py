"""The C ABI on the CPU: the library loads, exports every declared entry point, and its
host-only entry points behave (no device work here)."""
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1604_04026_amd as P

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "nmfkl.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(nmfkl_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    assert os.path.exists(P._LIB_PATH), "libnmfkl.so not built"
    out = subprocess.run(["nm", "-D", "--defined-only", P._LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (nmfkl_\w+)", out))
    missing = [s for s in declared_symbols() if s not in exported]
    assert not missing, missing
    assert set(P.EXPORTED_SYMBOLS) <= exported


def test_library_loads_and_binds():
    lib = P.load()
    for s in declared_symbols():
        assert hasattr(lib, s)


def test_params_default():
    p = P.nmfkl_params_default()
    assert (p.eps_x, p.t_max, p.j_max, p.guard, p.literal_break) == (0.1, 16, 8, 1, 0)
    assert p.eps_log == 1e-10 and p.eps_g == 1e-5 and p.foldin_max_passes == 200
    assert p.refresh_model == 0 and p.collect_stats == 0 and p.collect_timings == 0


def test_permutation_matches_oracle_and_numpy_stream(orc):
    for r in (1, 2, 10, 50, 100, 128):
        for t in (0, 1, 7, 123456789):
            for stream in (0, 1):
                a = P.nmfkl_permutation(5, t, stream, r)
                assert np.array_equal(a, orc.permutation(5, t, stream, r))
                assert sorted(a.tolist()) == list(range(r))


def test_permutation_rejects_bad_r():
    for r in (0, -1, 129):
        with pytest.raises(P.NmfklError) as e:
            P.nmfkl_permutation(0, 0, 0, r)
        assert e.value.code == -1


def test_create_rejects_null_problem():
    import ctypes
    lib = P.load()
    out = ctypes.c_void_p()
    assert lib.nmfkl_create(None, None, None, ctypes.byref(out)) == -1
    assert out.value is None
    assert b"null" in lib.nmfkl_last_error(None)
    assert lib.nmfkl_create(None, None, None, None) == -1


def test_create_rejects_bad_shapes_before_device_work():
    import ctypes
    lib = P.load()
    out = ctypes.c_void_p()
    base = dict(n=10, m=10, r=4, nnz=0, csc_ptr=1, csc_idx=1, csc_val=1, csr_ptr=1, csr_idx=1,
                csr_val=1, W=1, F=1)
    for bad in (dict(n=0), dict(m=-1), dict(r=0), dict(r=129), dict(nnz=-5), dict(W=None),
                dict(nnz=3, csc_idx=None)):
        kw = dict(base)
        kw.update(bad)
        prob = P.NmfklProblem(**kw)
        assert lib.nmfkl_create(ctypes.byref(prob), None, None, ctypes.byref(out)) == -1, bad
    prm = P.nmfkl_params_default(t_max=0)
    prob = P.NmfklProblem(**base)
    assert lib.nmfkl_create(ctypes.byref(prob), ctypes.byref(prm), None, ctypes.byref(out)) == -1
    prm = P.nmfkl_params_default(alpha_W=-1.0)
    assert lib.nmfkl_create(ctypes.byref(prob), ctypes.byref(prm), None, ctypes.byref(out)) == -1


def test_null_handle_calls_fail_cleanly():
    import ctypes
    lib = P.load()
    assert lib.nmfkl_sweep_F(None, 0) == -1
    assert lib.nmfkl_sweep_W(None, 0) == -1
    assert lib.nmfkl_invalidate_model(None) == -1
    assert lib.nmfkl_objective_enqueue(None) == -1
    d = ctypes.c_double()
    assert lib.nmfkl_objective_read(None, ctypes.byref(d)) == -1
    assert lib.nmfkl_destroy(None) == -1
