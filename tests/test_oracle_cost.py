"""Pins of the expensive stencil evaluation S(k) (Sec. 2, load patterns of Sec. 4).

Every entry S_o(k) = S_o + sum_t z * sin(t a + j_o c) with z = +0 adds exact
signed zeros, so sweeps with any k must equal the k = 0 sweeps bit for bit, for
fixed k and for k running over the mesh.  The same sweeps with a nonzero z
must differ (the added terms really reach the entries)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1810_04033_amd import inputs as I

CASES = [(2, 0, (9, 7)), (2, 1, (8, 6)), (3, 0, (5, 4, 6)), (3, 1, (6, 5, 4))]


def _case(dim, n, seed):
    shape = tuple(reversed(n))
    u = I.halo_array(I.uniform_field(I.stream_seed(seed, 1), shape))
    b = I.halo_array(I.uniform_field(I.stream_seed(seed, 2), shape))
    return u, b


@pytest.mark.parametrize("dim,stencil,n", CASES)
@pytest.mark.parametrize("kmax,hetero", [(0, 0), (3, 0), (17, 1), (100, 1)])
def test_cost_sweeps_equal_plain_sweeps(dim, stencil, n, kmax, hetero):
    u, b = _case(dim, n, 31)
    h = 1.0 / (max(n) + 1)
    ref = u.copy()
    O.gs_sweeps(ref, b, 2, dim=dim, stencil=stencil, h=h)
    got = u.copy()
    O.gs_sweeps_cost(got, b, 2, kmax, hetero, dim=dim, stencil=stencil, h=h)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("dim,stencil,n", CASES)
def test_nonzero_added_terms_change_the_iterate(dim, stencil, n):
    u, b = _case(dim, n, 32)
    h = 1.0 / (max(n) + 1)
    ref = u.copy()
    O.gs_sweeps(ref, b, 1, dim=dim, stencil=stencil, h=h)
    got = u.copy()
    O.gs_sweeps_cost(got, b, 1, 5, 0, dim=dim, stencil=stencil, h=h, z=1e-3)
    assert not np.array_equal(got, ref)
