"""V streamed from pinned host memory (params.out_of_core): the same method as the in-HBM
handle, with the model values computed per column/row from the tiles (Alg. 2's first step)
instead of carried.  Checked against the FP64 oracle (objective 1e-5 relative every sweep,
factors 1e-4) and against the in-HBM handle, with chunks small enough that every half-sweep
streams many of them."""
import ctypes

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


def corpus(n, m, r, seed, tag):
    ptr, idx, val = workloads.corpus(n, m, 80.0, 1.0, 2000, 1.1, 0.6, seed=seed, tag=tag)
    return workloads._problem(n, m, r, ptr, idx, val, seed, tag, {"name": f"corpus {n}x{m} r={r}"})


def run(prob, sweeps, prm, host_v):
    dev = P.upload_host_v(prob) if host_v else P.upload(prob)
    h = P.nmfkl_create(dev, prm)
    D = []
    for t in range(sweeps):
        P.nmfkl_sweep_F(h, t)
        P.nmfkl_sweep_W(h, t)
        D.append(P.nmfkl_objective(h))
    W, F = dev.W.cpu().numpy(), dev.F.cpu().numpy()
    P.nmfkl_destroy(h)
    return np.array(D), W, F


def test_out_of_core_trajectory_vs_oracle_and_in_hbm():
    prob = corpus(3000, 2000, 20, seed=0, tag=7)
    sweeps = 10
    prm = P.nmfkl_params_default(out_of_core=1, ooc_chunk_nnz=20000)
    D, W, F = run(prob, sweeps, prm, True)
    Wo, Fo, Do = oracle.run(prob, sweeps)
    rel = np.abs(D - Do) / Do
    Dh, Wh, Fh = run(prob, sweeps, P.nmfkl_params_default(), False)
    relh = np.abs(D - Dh) / Dh
    print(f"out-of-core ({int(prob.nnz / 20000) + 1}+ chunks per half): D rel vs oracle max {rel.max():.2e}, "
          f"vs in-HBM max {relh.max():.2e}; W {relf(W, Wo):.2e} F {relf(F, Fo):.2e}")
    assert rel.max() <= 1e-5 and relh.max() <= 1e-5
    assert relf(W, Wo) <= 1e-4 and relf(F, Fo) <= 1e-4


def test_out_of_core_long_rows_in_their_own_chunks():
    """Rows longer than the chunk budget (cooperative launches inside a chunk)."""
    n, m, r = 2000, 20000, 12
    prob = corpus(n, m, r, seed=0, tag=8)
    R = np.diff(prob.csr_ptr)
    assert R.max() > 4 * 4096
    t = 1
    ids = oracle.permutation(0, t, 0, r)
    Wo, _, _ = oracle.sweep_W(prob, prob.F0.astype(np.float64), prob.W0.astype(np.float64), ids)
    dev = P.upload_host_v(prob)
    h = P.nmfkl_create(dev, P.nmfkl_params_default(out_of_core=1, ooc_chunk_nnz=4096))
    P.nmfkl_sweep_W(h, t)
    Wg = dev.W.cpu().numpy()
    P.nmfkl_destroy(h)
    e = relf(Wg, Wo)
    print(f"out-of-core W-half with rows up to {R.max()} nonzeros (chunks of 4096): rel {e:.2e}")
    assert e <= 1e-4


def test_out_of_core_validates_on_the_host():
    prob = corpus(500, 400, 8, seed=2, tag=9)
    prob.csr_val = prob.csr_val.copy()
    k = int(np.argmax(prob.csr_val != prob.csr_val[0]))
    prob.csr_val[0], prob.csr_val[k] = prob.csr_val[k], prob.csr_val[0]
    dev = P.upload_host_v(prob)
    with pytest.raises(P.NmfklError) as ei:
        P.nmfkl_create(dev, P.nmfkl_params_default(out_of_core=1))
    assert ei.value.code == -1 and "transpose" in ei.value.message


def test_out_of_core_refuses_device_v_and_in_hbm_refuses_host_v():
    prob = corpus(500, 400, 8, seed=2, tag=9)
    for host_v, ooc in ((False, 1), (True, 0)):
        dev = P.upload_host_v(prob) if host_v else P.upload(prob)
        out = ctypes.c_void_p()
        st = dev.struct()
        prm = P.nmfkl_params_default(out_of_core=ooc)
        rc = P.load().nmfkl_create(ctypes.byref(st), ctypes.byref(prm), None, ctypes.byref(out))
        assert rc == -1 and not out.value, (host_v, ooc)
