"""FP32 sweeps inside FP64 iterative refinement: GPU against the oracle.

Parity: a fixed number of refinement steps on the GPU and in the oracle (same
scale rule, same inner sweep count) give the same iterate to 1e-13.
Convergence: the GPU reaches 1e-10 relative residual, measured by the oracle's
own FP64 residual of the GPU's final iterate.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_04033_amd import colsten as C
from paper_1810_04033_amd import inputs as I
from paper_1810_04033_amd import solve as S

import gpu_util as G

pytestmark = pytest.mark.gpu


def _grids(b_host, dim, st, h):
    n = tuple(reversed([s - 2 for s in b_host.shape]))
    x = C.empty_grid(n)
    b = C.empty_grid(n)
    b.copy_(torch.from_numpy(b_host))
    e = C.empty_grid(n, dtype=torch.float32)
    r32 = C.empty_grid(n, dtype=torch.float32)
    g64 = C.Grid(x, b, dim=dim, stencil=st, h=h)
    g32 = C.Grid(e, r32, dim=dim, stencil=st, h=h)
    return g64, g32


@pytest.mark.parametrize("dim,n,st", [(3, (24, 20, 16), C.CS_FD), (3, (24, 20, 16), C.CS_Q1),
                                      (2, (40, 30), C.CS_FD), (2, (33, 17), C.CS_Q1),
                                      (3, (65, 9, 10), C.CS_Q1)])
@pytest.mark.parametrize("inner", [7, 20])
def test_refinement_steps_match_oracle(dim, n, st, inner):
    h = 1.0 / (max(n) + 1)
    b_host = I.halo_array(I.uniform_field(31, tuple(reversed(n))))
    g64, g32 = _grids(b_host, dim, st, h)
    tmp32 = C.grid_like(g32.u)
    res = S.ir_solve(g64, g32, 0.0, inner_sweeps=inner, tmp32=tmp32, max_outer=4)
    x_ref, hist_ref, it_ref = O.ir_solve(b_host, 0.0, dim=dim, stencil=st, h=h,
                                         inner_sweeps=inner, max_outer=4)
    assert res.outer == it_ref == 4
    assert G.relmax(G.download(g64.u), x_ref) <= 1e-13
    np.testing.assert_allclose(res.history, hist_ref, rtol=1e-11)
    assert hist_ref[-1] < hist_ref[0]


@pytest.mark.parametrize("st", [C.CS_FD, C.CS_Q1])
def test_refinement_reaches_1e10_in_fp64(st):
    n = (32, 32, 32)
    h = 1.0 / 33
    b_host = I.halo_array(I.uniform_field(32, n))
    g64, g32 = _grids(b_host, 3, st, h)
    res = S.ir_solve(g64, g32, 1e-10, inner_sweeps=50, tmp32=C.grid_like(g32.u), max_outer=2000)
    assert res.converged and res.rel_residual <= 1e-10
    x = G.download(g64.u)
    norms = O.residual(x, b_host, dim=3, stencil=st, h=h)
    assert norms[0] / norms[2] <= 1e-10


def test_refinement_matches_plain_fp64_solution():
    """The refined FP32-sweep solution and plain FP64 sweeps converge to the
    same discrete solution (both to 1e-10 relative residual)."""
    n = (24, 24, 24)
    h = 1.0 / 25
    b_host = I.halo_array(I.uniform_field(33, n))
    g64, g32 = _grids(b_host, 3, C.CS_Q1, h)
    S.ir_solve(g64, g32, 1e-10, inner_sweeps=40, tmp32=C.grid_like(g32.u), max_outer=2000)
    u = C.empty_grid(n)
    b = C.empty_grid(n)
    b.copy_(torch.from_numpy(b_host))
    gp = C.Grid(u, b, dim=3, stencil=C.CS_Q1, h=h)
    r = S.gs_solve(gp, 1e-10, check_every=20, tmp=C.grid_like(u))
    assert r.converged
    assert G.relmax(G.download(g64.u), G.download(u)) <= 1e-8


def test_refinement_rejects_bad_arguments():
    b_host = I.halo_array(I.uniform_field(34, (8, 8, 8)))
    g64, g32 = _grids(b_host, 3, C.CS_FD, 1.0 / 9)
    norms = torch.zeros(3, dtype=torch.float64, device="cuda")
    for scale in (3.0, 0.0, -2.0, float("inf")):
        with pytest.raises(C.ColstenError):
            C.cs_ir_residual(g64.handle, g32.handle, scale, norms.data_ptr())
    with pytest.raises(C.ColstenError):
        C.cs_ir_residual(g32.handle, g64.handle, 1.0, norms.data_ptr())
    other = C.Grid(C.empty_grid((8, 8, 8), dtype=torch.float32),
                   C.empty_grid((8, 8, 8), dtype=torch.float32), dim=3, stencil=C.CS_Q1, h=1.0 / 9)
    with pytest.raises(C.ColstenError):
        C.cs_ir_update(g64.handle, other.handle, 1.0)


def test_config_refinement_512_full_size():
    """The mixed-precision workload at its full size (512^3, 27-point,
    Fourier + noise RHS of seed 4), in the launch configuration the benchmark
    times (fused sweeps with work arrays): one FP64 sweep, and one refinement
    step with one FP32 inner sweep, element by element against the oracle."""
    n, h = 512, 1.0 / 513
    st = C.CS_Q1
    b_host = I.halo_array(I.fourier_field(4, n))
    # FP64 fused sweep from u0 = 0
    g64, g32 = _grids(b_host, 3, st, h)
    tmp = C.grid_like(g64.u)
    g64.gs(1, tmp=tmp)
    torch.cuda.synchronize()
    uo = np.zeros_like(b_host)
    O.gs_sweeps(uo, b_host, 1, dim=3, stencil=st, h=h)
    assert G.relmax(G.download(g64.u), uo) <= 1e-13
    del tmp, uo
    # one refinement step: FP64 residual and scaled FP32 copy, one FP32 sweep, FP64 update
    g64.u.zero_()
    tmp32 = C.grid_like(g32.u)
    res = S.ir_solve(g64, g32, 0.0, inner_sweeps=1, tmp32=tmp32, max_outer=1)
    x_ref, hist_ref, it_ref = O.ir_solve(b_host, 0.0, dim=3, stencil=st, h=h,
                                         inner_sweeps=1, max_outer=1)
    assert res.outer == it_ref == 1
    assert G.relmax(G.download(g64.u), x_ref) <= 1e-13
    np.testing.assert_allclose(res.history, hist_ref, rtol=1e-11)
