"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host code, gcc) and
driven through its whole interface on small problems in a child process: every array access
of the C oracle stays in bounds and no undefined behaviour occurs (a sanitizer report makes
the child exit non-zero)."""
import os
import subprocess
import sys
import textwrap

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                           "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fPIC", "-shared", "-o", lib, os.path.join(ROOT, "oracle", "nmfkl_oracle.c"), "-lm"])
    script = textwrap.dedent(f"""
        import sys
        sys.path.insert(0, {ROOT!r})
        import numpy as np
        import oracle
        from paper_1604_04026_amd import workloads
        lib = oracle.load({lib!r})
        for prob in (workloads.config(0, seed=0), workloads.config(0, seed=3)):
            W, F = prob.W0.astype(np.float64), prob.F0.astype(np.float64)
            for t in range(2):
                ids = oracle.permutation(0, t, 0, prob.r)
                F, _, _ = oracle.sweep_F(prob, W, F, ids, lib=lib)
                W, _, _ = oracle.sweep_W(prob, F, W, ids, lib=lib)
            D = oracle.objective(prob, W, F, lib=lib)
            assert np.isfinite(D) and D >= 0
            # fold-in of a few documents over words whose rows of W are not all zero, one
            # document empty
            words = np.flatnonzero(W.sum(axis=1) > 0).astype(np.int32)
            ptr = np.array([0, 3, 3, 7], np.int64)
            idx = np.concatenate([np.sort(words[[1, 5, 9]]), np.sort(words[[2, 4, 6, 8]])])
            cnt = np.array([1, 2, 1, 3, 1, 1, 2], np.float64)
            Fd, passes, kl, _ = oracle.foldin(W, ptr, idx, cnt, lib=lib)
            assert Fd.shape == (3, prob.r) and np.all(np.isfinite(kl))
            sumW = W.sum(axis=0)
            assert np.isfinite(oracle.column_kl(idx[:3], cnt[:3], W, sumW, Fd[0], lib=lib))
        print("sanitized oracle ok")
    """)
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "sanitized oracle ok" in r.stdout, (r.stdout[-2000:] + r.stderr[-4000:])
