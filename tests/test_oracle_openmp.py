"""The oracle built with OpenMP -- one parallel loop per colour, the paper's
BSP colouring (Sec. 3) -- gives the sequential oracle's iterates bit for bit:
the points of one colour, and all points of a Jacobi sweep, are updated
independently, so the order of the parallel loop cannot matter."""
import os

import numpy as np
import pytest

from oracle import oracle as O


def _case(dim, n, seed):
    rng = np.random.default_rng(seed)
    shape = tuple(s + 2 for s in reversed(n))
    return rng.uniform(-1, 1, shape), rng.uniform(-1, 1, shape)


@pytest.fixture(autouse=True)
def _threads():
    old = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "4"
    yield
    O.set_openmp(False)
    if old is None:
        os.environ.pop("OMP_NUM_THREADS", None)
    else:
        os.environ["OMP_NUM_THREADS"] = old


@pytest.mark.parametrize("dim,n", [(2, (37, 29)), (3, (17, 13, 11)), (3, (8, 30, 5))])
@pytest.mark.parametrize("st", [O.FD, O.Q1])
@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_openmp_oracle_bitwise(dim, n, st, dt):
    u, b = _case(dim, n, 7 + dim + st)
    u, b = u.astype(dt), b.astype(dt)
    h = 1.0 / (max(n) + 1)
    res = {}
    for omp in (False, True):
        O.set_openmp(omp)
        ug, uj = u.copy(), u.copy()
        O.gs_sweeps(ug, b, 3, dim=dim, stencil=st, h=h, parity=1)
        O.jacobi_sweeps(uj, b, 3, 0.7, dim=dim, stencil=st, h=h)
        res[omp] = (ug, uj)
    O.set_openmp(False)
    assert np.array_equal(res[False][0], res[True][0])
    assert np.array_equal(res[False][1], res[True][1])
