"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these tests compares the oracle with itself or retypes its formulas:
the references are the paper's printed stencils and Algorithm 1 (golden
fixtures), a dense brute force assembled from textbook Kronecker products,
element assembly by Gauss quadrature, closed-form eigenpairs and spectral radii,
exactness on polynomials, and SPD-energy and order-invariance properties.
"""
import os

import numpy as np
import pytest
from fractions import Fraction

from oracle import oracle as O
from paper_1810_04033_amd import inputs as I

import bruteforce as BF

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rand_interior(seed, shape):
    return I.uniform_field(seed, shape)


def _halo(interior, pitch=None, halo=None):
    a = I.halo_array(interior, pitch=pitch)
    if halo is not None:
        fill = halo(a)
        a[...] = fill
    return a


def _relmax(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


# --------------------------------------------------------------------------
# Stencil entries
# --------------------------------------------------------------------------

def _read_fig1():
    out, cur = {}, None
    for line in open(os.path.join(GOLD, "fig1_stencils.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line in ("fd5", "q1_9"):
            cur = out.setdefault(line, [])
            continue
        cur.append([float(Fraction(t)) for t in line.split()])
    return {k: np.array(v) for k, v in out.items()}


def _stencil_by_delta(dim, stencil):
    """Apply the oracle's S to a unit impulse; read back the 3^d stencil."""
    n = 5
    shape = (n,) * dim
    u = I.halo_array(np.zeros(shape))
    c = (n // 2 + 1,) * dim
    u[c] = 1.0
    su = O.apply_stencil(u, dim=dim, stencil=stencil)
    sl = tuple(slice(ci - 1, ci + 2) for ci in c)
    return su[sl]


def test_fd5_and_q1_9_match_fig1():
    fig = _read_fig1()
    np.testing.assert_array_equal(_stencil_by_delta(2, O.FD), fig["fd5"])
    assert np.max(np.abs(_stencil_by_delta(2, O.Q1) - fig["q1_9"])) <= 4e-16


def _q1_element_stiffness(dim):
    """K_ab = int_[0,1]^d grad phi_a . grad phi_b by 2-point Gauss quadrature
    (exact for the products of d-linear gradients)."""
    g = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    nv = 1 << dim
    k = np.zeros((nv, nv))
    for qp in np.ndindex(*(2,) * dim):
        x = [g[t] for t in qp]
        grads = np.zeros((nv, dim))
        for a in range(nv):
            bits = [(a >> m) & 1 for m in range(dim)]
            for m in range(dim):
                val = 1.0
                for mm in range(dim):
                    if mm == m:
                        val *= 1.0 if bits[mm] else -1.0
                    else:
                        val *= x[mm] if bits[mm] else 1.0 - x[mm]
                grads[a, m] = val
        k += grads @ grads.T / (2 ** dim)
    return k


def _assembled_vertex_stencil(dim):
    kref = _q1_element_stiffness(dim)
    st = np.zeros((3,) * dim)
    nv = 1 << dim
    # vertex at the origin; the 2^d cells around it have lower corners in {-1,0}^d
    for cell in np.ndindex(*(2,) * dim):
        lo = [c - 1 for c in cell]
        a = sum(((0 - lo[m]) & 1) << m for m in range(dim))
        for b in range(nv):
            off = tuple(lo[m] + ((b >> m) & 1) for m in range(dim))
            st[tuple(reversed([o + 1 for o in off]))] += kref[a, b]
    return st


@pytest.mark.parametrize("dim", [2, 3])
def test_q1_stencil_equals_element_assembly(dim):
    st = _assembled_vertex_stencil(dim)
    got = _stencil_by_delta(dim, O.Q1)
    assert np.max(np.abs(got - st)) <= 1e-15
    if dim == 3:
        # faces of the trilinear stencil vanish; edges -1/6, corners -1/12
        assert abs(st[1, 1, 0]) < 1e-15 and abs(st[1, 0, 0] + 1 / 6) < 1e-15
        assert abs(st[0, 0, 0] + 1 / 12) < 1e-15 and abs(st[1, 1, 1] - 8 / 3) < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_element_stiffness_matches_oracle_kref(dim):
    k = _q1_element_stiffness(dim)
    for a in range(1 << dim):
        for b in range(1 << dim):
            nd = bin(a ^ b).count("1")
            assert abs(k[a, b] - O.q1_kref(dim, nd)) < 1e-15


@pytest.mark.parametrize("dim,shape", [(2, (7, 5)), (3, (5, 4, 3))])
def test_cellwise_q1_equals_stencil_form(dim, shape):
    u = _halo(_rand_interior(11, shape))
    u[0] = 0.3  # nonzero halo face
    a = O.apply_stencil(u, dim=dim, stencil=O.Q1)
    c = O.q1_apply_cellwise(u, dim=dim)
    ai, ci = O.interior(a), O.interior(c)
    assert _relmax(ci, ai) <= 1e-15
    # the same accumulation in 2^d cell-colour passes (different summation order)
    cc = O.interior(O.q1_apply_cellwise_coloured(u, dim=dim))
    assert _relmax(cc, ai) <= 1e-15


@pytest.mark.parametrize("dim,shape", [(2, (6, 7)), (3, (4, 5, 6))])
def test_cell_colours_share_no_vertex(dim, shape):
    # cells whose lower corners have the same parities are at least two apart
    # along some axis, so their vertex sets are disjoint
    import itertools
    rng = [range(0, n + 1) for n in shape]
    seen = {}
    for corner in itertools.product(*rng):
        col = sum((c & 1) << m for m, c in enumerate(corner))
        for off in itertools.product((0, 1), repeat=dim):
            v = tuple(c + o for c, o in zip(corner, off))
            assert (col, v) not in seen, (corner, seen.get((col, v)))
            seen[(col, v)] = corner


# --------------------------------------------------------------------------
# Colours
# --------------------------------------------------------------------------

def test_parity_one_reproduces_algorithm1_order():
    want = {0: set(), 1: set()}
    for line in open(os.path.join(GOLD, "alg1_red_black_n5.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        head, xs = line.split(":")
        c = int(head.split()[0][2:])
        y = int(head.split()[1][2:])
        for x in xs.split():
            want[c].add((int(x), y))
    for c in (0, 1):
        got = {(x, y) for y in range(1, 6) for x in range(1, 6) if O.colour(O.FD, 2, 1, x, y) == c}
        assert got == want[c]
    # parity 0 (the prose's greedy construction) puts the first point in colour 0
    assert O.colour(O.FD, 2, 0, 1, 1) == 0 and O.colour(O.FD, 3, 0, 1, 1, 1) == 0


def test_colouring_validity():
    assert O.colouring_valid(O.FD, 2, 6) and O.colouring_valid(O.FD, 3, 5)
    assert O.colouring_valid(O.Q1, 2, 6) and O.colouring_valid(O.Q1, 3, 5)
    # red-black does not resolve the races of the 3^d-point stencils
    assert not O.colouring_valid(O.Q1, 2, 6, force_red_black=True)
    assert not O.colouring_valid(O.Q1, 3, 5, force_red_black=True)
    assert O.num_colours(O.FD, 3) == 2 and O.num_colours(O.Q1, 2) == 4 and O.num_colours(O.Q1, 3) == 8


def test_colour_classes_have_near_equal_size():
    # Sec. 3: each of the c passes updates about N^d / c cells
    for stencil, dim, n in ((O.FD, 2, 9), (O.Q1, 2, 9), (O.FD, 3, 5), (O.Q1, 3, 5)):
        nc = O.num_colours(stencil, dim)
        counts = np.zeros(nc, dtype=int)
        for idx in np.ndindex(*(n,) * dim):
            p = [t + 1 for t in reversed(idx)] + [1]
            counts[O.colour(stencil, dim, 0, p[0], p[1], p[2])] += 1
        assert counts.sum() == n ** dim
        assert counts.max() - counts.min() <= n ** (dim - 1)


# --------------------------------------------------------------------------
# Operator and residual
# --------------------------------------------------------------------------

CASES = [(2, O.FD), (2, O.Q1), (3, O.FD), (3, O.Q1)]


def _coords(a_shape, h):
    """Physical coordinates (x, y[, z]) of every point of a halo'd array."""
    dim = len(a_shape)
    axes = [np.arange(s) * h for s in a_shape]
    mesh = np.meshgrid(*axes, indexing="ij")
    return list(reversed(mesh))  # x first


@pytest.mark.parametrize("dim,stencil", CASES)
def test_constants_and_linears_annihilated(dim, stencil):
    shape = (6, 5, 4)[:dim][::-1]
    h = 1.0 / 7
    for coeff in ([1.0] + [0.0] * dim, [0.25, 1.0, -2.0, 0.5][:dim + 1]):
        u = I.halo_array(np.zeros(shape))
        xs = _coords(u.shape, h)
        u[...] = coeff[0] + sum(c * x for c, x in zip(coeff[1:], xs))
        su = O.interior(O.apply_stencil(u, dim=dim, stencil=stencil))
        assert np.max(np.abs(su)) <= 1e-14


@pytest.mark.parametrize("dim,stencil", CASES)
def test_quadratic_gives_minus_2d_exactly_with_unit_spacing(dim, stencil):
    shape = (6, 5, 4)[:dim][::-1]
    u = I.halo_array(np.zeros(shape))
    xs = _coords(u.shape, 1.0)
    u[...] = sum(x * x for x in xs)
    b = I.halo_array(np.full(shape, -2.0 * dim))
    norms = O.residual(u, b, dim=dim, stencil=stencil, h=1.0)
    tol = 0.0 if stencil == O.FD else 1e-12
    assert norms[1] <= tol


def _closed_form_lambda(dim, stencil, ks, ns):
    c = [np.cos(k * np.pi / (n + 1)) for k, n in zip(ks, ns)]
    if stencil == O.FD:
        return sum(2.0 * (1.0 - cm) for cm in c)
    if dim == 2:
        return (2.0 / 3.0) * ((1 - c[0]) * (2 + c[1]) + (1 - c[1]) * (2 + c[0]))
    return (2.0 / 9.0) * ((1 - c[0]) * (2 + c[1]) * (2 + c[2]) + (1 - c[1]) * (2 + c[2]) * (2 + c[0])
                          + (1 - c[2]) * (2 + c[0]) * (2 + c[1]))


def _sine_mode(dim, ks, n):
    """prod_m sin(k_m pi i_m / (n+1)) on the halo'd cube grid (zero halo)."""
    u = I.halo_array(np.zeros((n,) * dim))
    idx = list(reversed(np.meshgrid(*[np.arange(n + 2)] * dim, indexing="ij")))
    val = np.ones(u.shape)
    for m in range(dim):
        val = val * np.sin(ks[m] * np.pi * idx[m] / (n + 1))
    u[...] = val
    return u


@pytest.mark.parametrize("dim,stencil", CASES)
def test_sine_modes_are_eigenvectors(dim, stencil):
    n = 9
    h = 1.0 / (n + 1)
    for ks in ([1, 1, 1][:dim], [2, 5, 3][:dim], [9, 1, 4][:dim]):
        u = _sine_mode(dim, ks, n)
        lam = _closed_form_lambda(dim, stencil, ks, [n] * dim)
        b = I.halo_array(np.zeros((n,) * dim))
        norms, r = O.residual(u, b, dim=dim, stencil=stencil, h=h, want_r=True)
        want = -lam / (h * h) * O.interior(u)
        assert _relmax(O.interior(r), want) <= 1e-12


@pytest.mark.parametrize("dim,stencil", CASES)
def test_residual_matches_dense(dim, stencil):
    n = (5, 4, 3)[:dim]
    h = 1.0 / 6
    u = _halo(_rand_interior(3, n[::-1]))
    u[..., 0] = 0.7  # nonzero Dirichlet values on one face
    b = _halo(_rand_interior(4, n[::-1]))
    norms, r = O.residual(u, b, dim=dim, stencil=stencil, h=h, want_r=True)
    rd = BF.residual(u.ravel(), O.interior(b).ravel(), dim, stencil, n, h)
    assert _relmax(O.interior(r).ravel(), rd) <= 1e-13
    assert abs(norms[0] - np.linalg.norm(rd)) <= 1e-12 * np.linalg.norm(rd)
    assert abs(norms[1] - np.max(np.abs(rd))) <= 1e-12 * np.max(np.abs(rd))
    assert abs(norms[2] - np.linalg.norm(O.interior(b))) <= 1e-14 * norms[2]


# --------------------------------------------------------------------------
# Gauss-Seidel colour passes and sweeps
# --------------------------------------------------------------------------

GS_SHAPES = [
    (2, O.FD, (7, 5)), (2, O.Q1, (6, 7)), (2, O.FD, (1, 1)), (2, O.Q1, (3, 2)),
    (3, O.FD, (5, 4, 3)), (3, O.Q1, (4, 5, 3)), (3, O.Q1, (2, 2, 2)), (3, O.FD, (1, 2, 3)),
]


@pytest.mark.parametrize("dim,stencil,n", GS_SHAPES)
@pytest.mark.parametrize("parity", [0, 1])
def test_gs_sweep_matches_dense_triangular_solve(dim, stencil, n, parity):
    h = 1.0 / (max(n) + 1)
    u = _halo(_rand_interior(5, n[::-1]))
    u[0] = -0.4  # nonzero boundary values on one face
    b = _halo(_rand_interior(6, n[::-1]))
    ref = u.ravel().copy()
    for _ in range(3):
        ref = BF.gs_sweep(ref, O.interior(b).ravel(), dim, stencil, n, h, parity)
    O.gs_sweeps(u, b, 3, dim=dim, stencil=stencil, h=h, parity=parity)
    assert _relmax(u.ravel(), ref) <= 1e-14


@pytest.mark.parametrize("dim,stencil,n", GS_SHAPES)
def test_lexicographic_sweep_matches_dense_triangular_solve(dim, stencil, n):
    # Sec. 3's task graph keeps the sequential issue order: natural-ordering GS
    h = 1.0 / (max(n) + 1)
    u = _halo(_rand_interior(15, n[::-1]))
    u[0] = 0.3
    b = _halo(_rand_interior(16, n[::-1]))
    ref = u.ravel().copy()
    for _ in range(3):
        ref = BF.gs_sweep_lex(ref, O.interior(b).ravel(), dim, stencil, n, h)
    O.lex_sweeps(u, b, 3, dim=dim, stencil=stencil, h=h)
    assert _relmax(u.ravel(), ref) <= 1e-14


@pytest.mark.parametrize("dim,stencil,n", GS_SHAPES)
def test_lexicographic_and_coloured_iterates_differ(dim, stencil, n):
    if np.prod(n) < 4 or (stencil == O.Q1 and max(n) <= 2):
        # with every point its own colour, colour order is the natural order
        pytest.skip("the orderings coincide on this grid")
    h = 1.0 / (max(n) + 1)
    u = _halo(_rand_interior(17, n[::-1]))
    b = _halo(_rand_interior(18, n[::-1]))
    lex, col = u.copy(), u.copy()
    O.lex_sweeps(lex, b, 1, dim=dim, stencil=stencil, h=h)
    O.gs_sweeps(col, b, 1, dim=dim, stencil=stencil, h=h)
    assert not np.array_equal(lex, col)


@pytest.mark.parametrize("dim,stencil", CASES)
def test_order_inside_a_colour_does_not_matter(dim, stencil):
    n = (6, 5, 4)[:dim]
    h = 1.0 / 7
    u0 = _halo(_rand_interior(7, n[::-1]))
    b = _halo(_rand_interior(8, n[::-1]))
    rng = np.random.default_rng(0)
    u1, u2 = u0.copy(), u0.copy()
    strides = [1, u0.strides[-2] // 8] + ([u0.strides[-3] // 8] if dim == 3 else [])
    for c in range(O.num_colours(stencil, dim)):
        O.colour_pass(u1, b, c, dim=dim, stencil=stencil, h=h)
        pts = []
        for idx in np.ndindex(*n[::-1]):
            p = [t + 1 for t in reversed(idx)]
            pc = O.colour(stencil, dim, 0, p[0], p[1], p[2] if dim == 3 else 1)
            if pc == c:
                pts.append(sum(pp * s for pp, s in zip(p, strides)))
        pts = np.array(pts, dtype=np.int64)
        rng.shuffle(pts)
        O.update_points(u2, b, pts, dim=dim, stencil=stencil, h=h)
        assert np.array_equal(u1, u2)


@pytest.mark.parametrize("dim,stencil", CASES)
def test_energy_never_increases(dim, stencil):
    n = (5, 4, 3)[:dim]
    h = 1.0 / 6
    a_ii, _, _, _ = BF.split(dim, stencil, n)
    u = _halo(_rand_interior(9, n[::-1]))
    b = _halo(_rand_interior(10, n[::-1]))
    bi = O.interior(b).ravel() * h * h

    def energy():
        x = O.interior(u).ravel()
        return 0.5 * x @ a_ii @ x - bi @ x

    e = energy()
    for _ in range(4):
        for c in range(O.num_colours(stencil, dim)):
            O.colour_pass(u, b, c, dim=dim, stencil=stencil, h=h)
            e2 = energy()
            assert e2 <= e + 1e-15 * abs(e)
            e = e2


@pytest.mark.parametrize("dim,stencil", CASES)
def test_single_point_grid(dim, stencil):
    h = 0.5
    u = I.halo_array(np.zeros((1,) * dim))
    b = I.halo_array(np.full((1,) * dim, 0.75))
    O.gs_sweeps(u, b, 1, dim=dim, stencil=stencil, h=h)
    s0 = 2.0 * dim if stencil == O.FD else 8.0 / 3.0
    assert abs(O.interior(u).item() - 0.25 * 0.75 / s0) <= 1e-16


@pytest.mark.parametrize("dim,stencil", CASES)
def test_quadratic_is_a_fixed_point(dim, stencil):
    shape = (5, 4, 3)[:dim][::-1]
    h = 1.0 / 8
    u = I.halo_array(np.zeros(shape))
    xs = _coords(u.shape, h)
    u[...] = sum(x * x for x in xs)
    ref = u.copy()
    b = I.halo_array(np.full(shape, -2.0 * dim))
    O.gs_sweeps(u, b, 2, dim=dim, stencil=stencil, h=h)
    assert np.max(np.abs(u - ref)) <= 1e-14


@pytest.mark.parametrize("dim,stencil", CASES)
def test_sweeps_converge_to_direct_solve(dim, stencil):
    n = (6, 5, 4)[:dim]
    h = 1.0 / 7
    a_ii, a_ib, cols, bcols = BF.split(dim, stencil, n)
    u = _halo(_rand_interior(12, n[::-1]))
    u[...] = 0.0
    b = _halo(_rand_interior(13, n[::-1]))
    exact = np.linalg.solve(a_ii, h * h * O.interior(b).ravel())
    O.gs_sweeps(u, b, 400, dim=dim, stencil=stencil, h=h)
    assert _relmax(O.interior(u).ravel(), exact) <= 1e-10


@pytest.mark.parametrize("dim,n", [(2, 15), (3, 7)])
def test_red_black_rate_is_cos_squared(dim, n):
    # Young: red-black ordering of the 2d+1 stencil is consistently ordered, so
    # the GS spectral radius is the square of Jacobi's, cos(pi h)^2.
    h = 1.0 / (n + 1)
    u = _halo(_rand_interior(14, (n,) * dim))
    b = I.halo_array(np.zeros((n,) * dim))
    O.gs_sweeps(u, b, 500, dim=dim, stencil=O.FD, h=h)
    n0 = np.linalg.norm(O.interior(u))
    O.gs_sweeps(u, b, 1, dim=dim, stencil=O.FD, h=h)
    rate = np.linalg.norm(O.interior(u)) / n0
    assert abs(rate - np.cos(np.pi * h) ** 2) <= 1e-9


# --------------------------------------------------------------------------
# Jacobi
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim,stencil", CASES)
@pytest.mark.parametrize("omega", [1.0, 2.0 / 3.0])
def test_jacobi_scales_sine_modes_by_closed_form(dim, stencil, omega):
    n = 9
    h = 1.0 / (n + 1)
    ks = [3, 1, 2][:dim]
    u = _sine_mode(dim, ks, n)
    u0 = O.interior(u).copy()
    b = I.halo_array(np.zeros((n,) * dim))
    O.jacobi_sweeps(u, b, 1, omega, dim=dim, stencil=stencil, h=h)
    s0 = 2.0 * dim if stencil == O.FD else 8.0 / 3.0
    mu = 1.0 - omega * _closed_form_lambda(dim, stencil, ks, [n] * dim) / s0
    assert _relmax(O.interior(u), mu * u0) <= 1e-13


@pytest.mark.parametrize("dim,stencil", CASES)
def test_jacobi_matches_dense(dim, stencil):
    n = (5, 4, 3)[:dim]
    h = 1.0 / 6
    u = _halo(_rand_interior(15, n[::-1]))
    u[..., -1] = 0.2
    b = _halo(_rand_interior(16, n[::-1]))
    ref = u.ravel().copy()
    for _ in range(3):
        ref = BF.jacobi_sweep(ref, O.interior(b).ravel(), dim, stencil, n, h, 2.0 / 3.0)
    O.jacobi_sweeps(u, b, 3, 2.0 / 3.0, dim=dim, stencil=stencil, h=h)
    assert _relmax(u.ravel(), ref) <= 1e-14


def test_jacobi_rate_is_cos():
    n, dim = 15, 2
    h = 1.0 / (n + 1)
    u = _halo(_rand_interior(17, (n,) * dim))
    b = I.halo_array(np.zeros((n,) * dim))
    O.jacobi_sweeps(u, b, 600, 1.0, dim=dim, stencil=O.FD, h=h)
    # undamped Jacobi alternates sign on the +-cos(pi h) pair: use two steps
    n0 = np.linalg.norm(O.interior(u))
    O.jacobi_sweeps(u, b, 2, 1.0, dim=dim, stencil=O.FD, h=h)
    rate = np.sqrt(np.linalg.norm(O.interior(u)) / n0)
    assert abs(rate - np.cos(np.pi * h)) <= 1e-9


# --------------------------------------------------------------------------
# Layout, precision, refinement
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim,stencil", CASES)
def test_padded_pitch_gives_identical_bits(dim, stencil):
    n = (7, 5, 4)[:dim]
    h = 1.0 / 8
    it = _rand_interior(18, n[::-1])
    bt = _rand_interior(19, n[::-1])
    u1, b1 = I.halo_array(it), I.halo_array(bt)
    u2, b2 = I.halo_array(it, pitch=16), I.halo_array(bt, pitch=16)
    O.gs_sweeps(u1, b1, 3, dim=dim, stencil=stencil, h=h)
    O.gs_sweeps(u2, b2, 3, dim=dim, stencil=stencil, h=h)
    assert np.array_equal(u1, u2)


@pytest.mark.parametrize("dim,stencil", CASES)
def test_fp32_sweeps_track_fp64(dim, stencil):
    n = (9, 8, 7)[:dim]
    h = 1.0 / 10
    it = _rand_interior(20, n[::-1])
    bt = _rand_interior(21, n[::-1])
    u64, b64 = I.halo_array(it), I.halo_array(bt)
    u32 = I.halo_array(it, dtype=np.float32)
    b32 = I.halo_array(bt, dtype=np.float32)
    O.gs_sweeps(u64, b64, 10, dim=dim, stencil=stencil, h=h)
    O.gs_sweeps(u32, b32, 10, dim=dim, stencil=stencil, h=h)
    assert _relmax(u32.astype(np.float64), u64) <= 1e-5


def test_ir_reaches_tolerance_with_fp64_residual():
    n, dim = 12, 3
    h = 1.0 / (n + 1)
    b = I.halo_array(_rand_interior(22, (n,) * dim))
    x, hist, it = O.ir_solve(b, 1e-10, dim=dim, stencil=O.Q1, h=h, inner_sweeps=40, max_outer=60)
    assert hist[-1] <= 1e-10 and it < 60
    norms = O.residual(x, b, dim=dim, stencil=O.Q1, h=h)
    assert norms[0] / norms[2] <= 1e-10
    # FP32 sweeps alone stall near single precision
    u32 = I.halo_array(np.zeros((n,) * dim), dtype=np.float32)
    b32 = b.astype(np.float32)
    O.gs_sweeps(u32, b32, 2000, dim=dim, stencil=O.Q1, h=h)
    n32 = O.residual(u32, b32, dim=dim, stencil=O.Q1, h=h)
    assert n32[0] / n32[2] > 1e-9


def test_splitmix64_reference_outputs():
    # published SplitMix64 outputs for state 0 (Steele, Lea & Flood 2014)
    v = I.splitmix64(0, np.arange(4, dtype=np.uint64))
    assert [int(x) for x in v] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                   0x06C45D188009454F, 0xF88BB8A8724C81EC]
    f = I.uniform_field(1, (3, 4))
    assert f.min() >= -1.0 and f.max() < 1.0
