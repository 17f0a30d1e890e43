"""Pins of the oracle's single-precision functions.

The FP32 colour sweeps, FP32 Jacobi sweeps, FP32 lexicographic sweeps and the
FP64 residual of an FP32 grid are the references of every FP32 parity test, so
each is pinned here against something other than the oracle's own FP32 code:
closed-form eigenvalues, the dense triangular solve of the brute-force module,
and the FP64 functions, which are themselves pinned by dense brute force and
closed forms.  Tolerances are FP32 rounding bounds.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1810_04033_amd import inputs as I

import bruteforce as BF

CASES = [(2, O.FD), (2, O.Q1), (3, O.FD), (3, O.Q1)]


def _relmax(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _halo32(interior, pitch=None):
    return I.halo_array(interior, pitch=pitch, dtype=np.float32)


def _closed_form_lambda(dim, stencil, ks, ns):
    """Eigenvalue of the dimensionless stencil on prod_m sin(k_m pi x_m)."""
    c = [np.cos(k * np.pi / (n + 1)) for k, n in zip(ks, ns)]
    if stencil == O.FD:
        return sum(2.0 * (1.0 - cm) for cm in c)
    if dim == 2:
        return (2.0 / 3.0) * ((1 - c[0]) * (2 + c[1]) + (1 - c[1]) * (2 + c[0]))
    return (2.0 / 9.0) * ((1 - c[0]) * (2 + c[1]) * (2 + c[2]) + (1 - c[1]) * (2 + c[2]) * (2 + c[0])
                          + (1 - c[2]) * (2 + c[0]) * (2 + c[1]))


def _sine_mode32(dim, ks, n):
    u = I.halo_array(np.zeros((n,) * dim), dtype=np.float32)
    idx = list(reversed(np.meshgrid(*[np.arange(n + 2)] * dim, indexing="ij")))
    val = np.ones(u.shape)
    for m in range(dim):
        val = val * np.sin(ks[m] * np.pi * idx[m] / (n + 1))
    u[...] = val.astype(np.float32)
    return u


# --------------------------------------------------------------------------
# Weighted Jacobi in FP32
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim,stencil", CASES)
@pytest.mark.parametrize("omega", [2.0 / 3.0, 0.8])
def test_fp32_jacobi_scales_sine_modes_by_closed_form(dim, stencil, omega):
    # one damped Jacobi step maps an eigenvector to mu u with
    # mu = 1 - omega lambda / S_0; in FP32 the image agrees to a few ulps
    n = 9
    h = 1.0 / (n + 1)
    for ks in ([3, 1, 2][:dim], [1, 1, 1][:dim]):
        u = _sine_mode32(dim, ks, n)
        u0 = O.interior(u).astype(np.float64)
        b = I.halo_array(np.zeros((n,) * dim), dtype=np.float32)
        O.jacobi_sweeps(u, b, 1, omega, dim=dim, stencil=stencil, h=h)
        s0 = 2.0 * dim if stencil == O.FD else 8.0 / 3.0
        mu = 1.0 - omega * _closed_form_lambda(dim, stencil, ks, [n] * dim) / s0
        assert _relmax(O.interior(u).astype(np.float64), mu * u0) <= 2e-6


@pytest.mark.parametrize("dim,stencil", CASES)
def test_fp32_jacobi_matches_dense(dim, stencil):
    n = (5, 4, 3)[:dim]
    h = 1.0 / 6
    it = I.uniform_field(31, n[::-1])
    bt = I.uniform_field(32, n[::-1])
    u = _halo32(it)
    u[..., -1] = 0.25  # nonzero Dirichlet values on one face
    b = _halo32(bt)
    ref = u.astype(np.float64).ravel()
    bi = O.interior(b).astype(np.float64).ravel()
    for _ in range(3):
        ref = BF.jacobi_sweep(ref, bi, dim, stencil, n, h, 2.0 / 3.0)
    O.jacobi_sweeps(u, b, 3, 2.0 / 3.0, dim=dim, stencil=stencil, h=h)
    assert _relmax(u.astype(np.float64).ravel(), ref) <= 1e-5


@pytest.mark.parametrize("dim,stencil", CASES)
def test_fp32_jacobi_tracks_fp64(dim, stencil):
    n = (9, 8, 7)[:dim]
    h = 1.0 / 10
    it = I.uniform_field(33, n[::-1])
    bt = I.uniform_field(34, n[::-1])
    u64, b64 = I.halo_array(it), I.halo_array(bt)
    u32, b32 = _halo32(it), _halo32(bt)
    O.jacobi_sweeps(u64, b64, 12, 2.0 / 3.0, dim=dim, stencil=stencil, h=h)
    O.jacobi_sweeps(u32, b32, 12, 2.0 / 3.0, dim=dim, stencil=stencil, h=h)
    assert _relmax(u32.astype(np.float64), u64) <= 1e-5


# --------------------------------------------------------------------------
# Lexicographic Gauss-Seidel in FP32
# --------------------------------------------------------------------------

LEX_SHAPES = [(2, O.FD, (7, 5)), (2, O.Q1, (6, 7)), (3, O.FD, (5, 4, 3)), (3, O.Q1, (4, 5, 3))]


@pytest.mark.parametrize("dim,stencil,n", LEX_SHAPES)
def test_fp32_lexicographic_sweep_matches_dense_triangular_solve(dim, stencil, n):
    # natural-ordering Gauss-Seidel as (D + L) u_new = h^2 b - A_IB g - U u_old
    h = 1.0 / (max(n) + 1)
    u = _halo32(I.uniform_field(35, n[::-1]))
    u[0] = 0.3
    b = _halo32(I.uniform_field(36, n[::-1]))
    ref = u.astype(np.float64).ravel()
    bi = O.interior(b).astype(np.float64).ravel()
    for _ in range(3):
        ref = BF.gs_sweep_lex(ref, bi, dim, stencil, n, h)
    O.lex_sweeps(u, b, 3, dim=dim, stencil=stencil, h=h)
    assert _relmax(u.astype(np.float64).ravel(), ref) <= 1e-5


@pytest.mark.parametrize("dim,stencil,n", LEX_SHAPES)
def test_fp32_lexicographic_sweep_tracks_fp64(dim, stencil, n):
    h = 1.0 / (max(n) + 1)
    it = I.uniform_field(37, n[::-1])
    bt = I.uniform_field(38, n[::-1])
    u64, b64 = I.halo_array(it), I.halo_array(bt)
    u32, b32 = _halo32(it), _halo32(bt)
    O.lex_sweeps(u64, b64, 8, dim=dim, stencil=stencil, h=h)
    O.lex_sweeps(u32, b32, 8, dim=dim, stencil=stencil, h=h)
    assert _relmax(u32.astype(np.float64), u64) <= 1e-5


# --------------------------------------------------------------------------
# FP64 residual of an FP32 grid
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dim,stencil", CASES)
@pytest.mark.parametrize("pitch", [None, 16])
def test_fp32_grid_residual_equals_fp64_residual_of_widened_values(dim, stencil, pitch):
    # widening binary32 to binary64 is exact, so the residual of the FP32 grid
    # evaluated in FP64 is the FP64 residual of the widened arrays, bit for bit
    n = (6, 5, 4)[:dim]
    h = 1.0 / 7
    u32 = _halo32(I.uniform_field(39, n[::-1]), pitch=pitch)
    u32[..., 0] = 0.5
    b32 = _halo32(I.uniform_field(40, n[::-1]), pitch=pitch)
    got = O.residual(u32, b32, dim=dim, stencil=stencil, h=h)
    u64 = I.halo_array(O.interior(u32).astype(np.float64), pitch=pitch)
    u64[...] = u32.astype(np.float64)
    b64 = I.halo_array(O.interior(b32).astype(np.float64), pitch=pitch)
    want = O.residual(u64, b64, dim=dim, stencil=stencil, h=h)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dim,stencil", CASES)
def test_fp32_grid_residual_matches_dense(dim, stencil):
    n = (5, 4, 3)[:dim]
    h = 1.0 / 6
    u32 = _halo32(I.uniform_field(41, n[::-1]))
    u32[..., 0] = 0.75
    b32 = _halo32(I.uniform_field(42, n[::-1]))
    norms = O.residual(u32, b32, dim=dim, stencil=stencil, h=h)
    rd = BF.residual(u32.astype(np.float64).ravel(), O.interior(b32).astype(np.float64).ravel(),
                     dim, stencil, n, h)
    assert abs(norms[0] - np.linalg.norm(rd)) <= 1e-12 * np.linalg.norm(rd)
    assert abs(norms[1] - np.max(np.abs(rd))) <= 1e-12 * np.max(np.abs(rd))
    bn = np.linalg.norm(O.interior(b32).astype(np.float64))
    assert abs(norms[2] - bn) <= 1e-14 * bn
