"""Pins of the oracle's multigrid V-cycle (the coloured sweep as smoother)
against facts of the transfers and of multigrid theory, not against the
oracle's own formulas:

* full weighting keeps constants and affine functions (weights sum to one,
  symmetric about the coarse point), exactly;
* d-linear interpolation reproduces d-linear functions, exactly;
* restriction is the adjoint of interpolation scaled by 2^-d;
* for the d-linear finite-element stencils the Galerkin product R A_h P is
  the same stencil on the grid of spacing 2h (element stiffness scales with
  h^(d-2));
* V(2,2)-cycles reduce the residual by a factor bounded away from one that
  does not grow with the grid (textbook multigrid convergence).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1810_04033_amd import inputs as I


def _zeros(n, pitch=None):
    return I.halo_array(np.zeros(tuple(reversed(n))), pitch=pitch)


def _index_grids(a, dim):
    """Index arrays (i, j[, k]) of every element of a halo'd array."""
    idx = np.indices(a.shape)
    return (idx[-1], idx[-2]) if dim == 2 else (idx[-1], idx[-2], idx[-3])


def _coarse(n):
    return tuple((v - 1) // 2 for v in n)


SHAPES = [(3, 3), (7, 5), (15, 31), (3, 3, 3), (7, 5, 9), (15, 7, 3)]


@pytest.mark.parametrize("n", SHAPES, ids=lambda p: "x".join(map(str, p)))
def test_restriction_keeps_constants(n):
    dim = len(n)
    r = _zeros(n, pitch=n[0] + 5)
    r[...] = 0.0
    r[(slice(1, -1),) * dim] = 0.8125
    # the halo of r is never read: fill it with something else
    r[(0,) * dim] = 99.0
    bc, uc = _zeros(_coarse(n)), _zeros(_coarse(n))
    uc[...] = 5.0
    O.restrict(r, bc, uc, dim=dim)
    inner = (slice(1, -1),) * dim
    assert np.all(bc[inner] == 0.8125)
    assert np.all(uc[inner] == 0.0)
    # halos untouched
    assert np.all(uc[0] == 5.0) and np.all(bc[0] == 0.0)


@pytest.mark.parametrize("n", SHAPES, ids=lambda p: "x".join(map(str, p)))
def test_restriction_keeps_affine_functions(n):
    # f = 3 + 2 i - 5 j (+ 7 k) in fine index units; at coarse point I the
    # weighted mean over the 3^d block around 2I is f(2I) exactly
    dim = len(n)
    r = _zeros(n)
    ij = _index_grids(r, dim)
    coef = (2.0, -5.0, 7.0)
    r[...] = 3.0 + sum(c * t for c, t in zip(coef, ij))
    bc, uc = _zeros(_coarse(n)), _zeros(_coarse(n))
    O.restrict(r, bc, uc, dim=dim)
    IJ = _index_grids(bc, dim)
    want = 3.0 + sum(c * 2 * t for c, t in zip(coef, IJ))
    inner = (slice(1, -1),) * dim
    assert np.array_equal(bc[inner], want[inner])


@pytest.mark.parametrize("n", SHAPES, ids=lambda p: "x".join(map(str, p)))
def test_interpolation_reproduces_multilinear_functions(n):
    # g(I, J, K) = 1 + 2I - J + 3K + IJ - 2JK + IJK (coarse units, halo
    # included); at fine point i its interpolant is g(i/2, j/2, k/2)
    dim = len(n)
    uc = _zeros(_coarse(n), pitch=_coarse(n)[0] + 3)
    if dim == 2:
        g = lambda x, y: 1 + 2 * x - y + 0.75 * x * y
    else:
        g = lambda x, y, z: 1 + 2 * x - y + 3 * z + x * y - 2 * y * z + x * y * z
    uc[...] = g(*[t.astype(np.float64) for t in _index_grids(uc, dim)])
    uf = _zeros(n)
    O.prolong_add(uc, uf, dim=dim)
    want = g(*[t / 2.0 for t in _index_grids(uf, dim)])
    inner = (slice(1, -1),) * dim
    assert np.array_equal(uf[inner], want[inner])
    assert np.all(uf[0] == 0.0)  # fine halo untouched


@pytest.mark.parametrize("n", [(15, 7), (31, 31), (7, 9, 5), (15, 15, 15)],
                         ids=lambda p: "x".join(map(str, p)))
def test_restriction_is_scaled_adjoint_of_interpolation(n):
    dim = len(n)
    r = I.halo_array(I.uniform_field(11, tuple(reversed(n))))
    v = I.halo_array(I.uniform_field(12, tuple(reversed(_coarse(n)))))  # zero halo
    bc, uc = _zeros(_coarse(n)), _zeros(_coarse(n))
    O.restrict(r, bc, uc, dim=dim)
    pv = _zeros(n)
    O.prolong_add(v, pv, dim=dim)
    lhs = float(np.sum(bc * v))
    rhs = float(np.sum(r[(slice(1, -1),) * dim] * pv[(slice(1, -1),) * dim])) / 2 ** dim
    assert abs(lhs - rhs) <= 1e-13 * abs(rhs)


@pytest.mark.parametrize("n", [(15, 31), (7, 7, 7), (15, 9, 5)], ids=lambda p: "x".join(map(str, p)))
def test_galerkin_product_of_d_linear_stencil(n):
    # R A_h P = A_2h for the Q1 stencils: with A = S / h^2 and K_h = h^(d-2) S
    # the element stiffness, P^T K_h P = K_2h gives R A_h P = A_2h, R = P^T/2^d
    dim = len(n)
    h = 1.0 / 64
    e = I.halo_array(I.uniform_field(13, tuple(reversed(_coarse(n)))))  # zero halo
    pe = _zeros(n)
    O.prolong_add(e, pe, dim=dim)
    y = O.apply_stencil(pe, dim=dim, stencil=O.Q1) / (h * h)
    bc, uc = _zeros(_coarse(n)), _zeros(_coarse(n))
    O.restrict(y, bc, uc, dim=dim)
    want = O.apply_stencil(e, dim=dim, stencil=O.Q1) / (2 * h) ** 2
    inner = (slice(1, -1),) * dim
    err = np.max(np.abs(bc[inner] - want[inner])) / np.max(np.abs(want[inner]))
    assert err <= 1e-12


def _factors(dim, n, stencil, cycles):
    h = 1.0 / (n + 1)
    b = I.halo_array(I.uniform_field(7, (n,) * dim))
    u = np.zeros_like(b)
    r = [O.residual(u, b, dim=dim, stencil=stencil, h=h)[0]]
    for _ in range(cycles):
        O.mg_vcycle(u, b, dim=dim, stencil=stencil, h=h)
        r.append(O.residual(u, b, dim=dim, stencil=stencil, h=h)[0])
    return [r[i + 1] / r[i] for i in range(1, cycles)]


@pytest.mark.parametrize("dim,stencil,bound", [(2, O.FD, 0.07), (2, O.Q1, 0.03),
                                               (3, O.FD, 0.12), (3, O.Q1, 0.03)])
def test_vcycle_converges_independently_of_h(dim, stencil, bound):
    # red-black / 2^d-colour Gauss-Seidel V(2,2)-cycles: each cycle cuts the
    # residual by a fixed factor well below one, the same on a finer grid
    n1, n2 = (31, 63) if dim == 2 else (15, 31)
    f1 = _factors(dim, n1, stencil, 5)
    f2 = _factors(dim, n2, stencil, 5)
    assert max(f1) <= bound and max(f2) <= bound
    # halving h leaves the factor about the same (plain sweeps: 1 - O(h^2))
    assert f2[-1] <= 1.35 * f1[-1]


def test_vcycle_without_coarser_grid_is_plain_sweeps():
    # an even size does not coarsen: the cycle is coarse_sweeps sweeps
    n = (8, 6, 5)
    h = 1.0 / 9
    b = I.halo_array(I.uniform_field(3, tuple(reversed(n))))
    u1, u2 = np.zeros_like(b), np.zeros_like(b)
    O.mg_vcycle(u1, b, dim=3, stencil=O.FD, h=h, coarse_sweeps=3)
    O.gs_sweeps(u2, b, 3, dim=3, stencil=O.FD, h=h)
    assert np.array_equal(u1, u2)


def test_transfers_reject_mismatched_sizes():
    with pytest.raises(ValueError):
        O.restrict(_zeros((7, 7)), _zeros((4, 3)), _zeros((4, 3)), dim=2)
    with pytest.raises(ValueError):
        O.prolong_add(_zeros((3, 3, 2)), _zeros((7, 7, 7)), dim=3)


def test_driver_and_oracle_coarsen_alike():
    # the GPU driver's level rule (host logic, no GPU) and the oracle's agree,
    # and sizes 2^m - 1 reach one point
    from paper_1810_04033_amd import mg as MG
    for n in [(1,), (3, 3), (7, 5), (8, 7), (15, 7, 31), (255, 255, 255), (2, 3, 3), (63, 127)]:
        assert MG.coarsens(n) == O.mg_coarsens(n)
    n, levels = (255, 255, 255), 1
    while MG.coarsens(n):
        n = tuple((v - 1) // 2 for v in n)
        levels += 1
    assert n == (1, 1, 1) and levels == 8
