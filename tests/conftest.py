import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.load()
    return oracle


def random_column(rng, n=12, r=4, L=None, density=0.6, scale=3.0):
    """A small dense-backed subproblem: A (n x r) >= 0 with some exact zeros, v >= 0 with
    nonzeros at a random subset of points, x >= 0 with some exact zeros."""
    A = rng.gamma(0.5, 1.0, size=(n, r))
    A[rng.random((n, r)) < 0.2] = 0.0
    dead = np.nonzero(A.sum(axis=1) == 0)[0]
    A[dead, rng.integers(0, r, dead.size)] = rng.gamma(0.5, 1.0, dead.size) + 0.1
    if L is None:
        L = max(1, int(density * n))
    idx = np.sort(rng.choice(n, size=L, replace=False)).astype(np.int32)
    v = np.floor(rng.gamma(1.0, scale, size=L)) + 1.0
    x = rng.gamma(0.7, 1.0, size=r)
    x[rng.random(r) < 0.3] = 0.0
    return A, idx, v, x
