"""Fused sweeps of 2D grids: several whole sweeps per launch on an LDS-resident
tile (up to 4 red-black or 2 four-colour sweeps; 32 x 32 or, on grids with a
tile per CU, 64 x 32 tiles).  Every sweep count from 1 to 9 (each split into
launches of 4, 2 and 1 sweeps) must give the oracle's
coloured iterate bit for bit, on grids of several tiles with ragged tails,
both stencils and colour parities, every layout, a random Dirichlet halo, FP64
and FP32; with one sweep per pass as well.  The same for the weighted Jacobi
sweeps (up to 8 per launch on small grids, 4 on large ones)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_04033_amd import colsten as C

import gpu_util as G

pytestmark = pytest.mark.gpu

NP = {torch.float64: np.float64, torch.float32: np.float32}
SHAPES = [(1, 1), (2, 3), (5, 7), (31, 33), (64, 3), (65, 33), (130, 70), (200, 97), (1030, 530)]


def _run(n, st, nsw, dt, layout, parity, mode, seed):
    u, b = G.case(2, n, seed=seed)
    h = 1.0 / (max(n) + 1)
    uo, bo = u.astype(NP[dt]), b.astype(NP[dt])
    O.gs_sweeps(uo, bo, nsw, dim=2, stencil=st, h=h, parity=parity)
    ug, bg = G.upload(u, dt, layout=layout), G.upload(b, dt, layout=layout)
    g = C.Grid(ug, bg, dim=2, stencil=st, h=h, parity=parity)
    g.set_pass_mode(mode)
    g.gs(nsw, tmp=C.grid_like(ug))
    torch.cuda.synchronize()
    return ug.detach().cpu().numpy(), uo


@pytest.mark.parametrize("n", SHAPES, ids=lambda p: "x".join(map(str, p)))
@pytest.mark.parametrize("st", [C.CS_FD, C.CS_Q1], ids=["fd", "q1"])
@pytest.mark.parametrize("nsw", list(range(1, 10)))
@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_fused2d_bitwise(n, st, nsw, dt):
    got, want = _run(n, st, nsw, dt, "aligned", nsw % 2, C.CS_PASS_AUTO, 1800 + nsw)
    assert np.array_equal(got, want), "max diff %g" % np.max(np.abs(got.astype(np.float64) - want))


@pytest.mark.parametrize("layout", ["compact", "odd"])
@pytest.mark.parametrize("st", [C.CS_FD, C.CS_Q1], ids=["fd", "q1"])
@pytest.mark.parametrize("mode", [C.CS_PASS_AUTO, C.CS_PASS_ONE], ids=["auto", "one"])
def test_fused2d_layouts_and_modes(layout, st, mode):
    got, want = _run((97, 45), st, 7, torch.float64, layout, 1, mode, 1900)
    assert np.array_equal(got, want)


def test_fused2d_sweeps_per_pass():
    u = C.empty_grid((256, 256))
    for st, per in ((C.CS_FD, 4), (C.CS_Q1, 2)):
        g = C.Grid(u, C.grid_like(u), dim=2, stencil=st, h=0.1)
        assert g.fused and g.sweeps_per_pass() == per
        assert g.sweeps_per_pass(jacobi=True) > 1
        g.set_pass_mode(C.CS_PASS_ONE)
        assert g.sweeps_per_pass() == 1 and g.sweeps_per_pass(jacobi=True) == 1
        g.close()


def _run_jacobi(n, st, nsw, dt, layout, mode, seed, omega=0.8):
    u, b = G.case(2, n, seed=seed)
    h = 1.0 / (max(n) + 1)
    uo, bo = u.astype(NP[dt]), b.astype(NP[dt])
    O.jacobi_sweeps(uo, bo, nsw, omega, dim=2, stencil=st, h=h)
    ug, bg = G.upload(u, dt, layout=layout), G.upload(b, dt, layout=layout)
    g = C.Grid(ug, bg, dim=2, stencil=st, h=h)
    g.set_pass_mode(mode)
    g.jacobi(omega, nsw, C.grid_like(ug))
    torch.cuda.synchronize()
    return ug.detach().cpu().numpy(), uo


@pytest.mark.parametrize("n", SHAPES, ids=lambda p: "x".join(map(str, p)))
@pytest.mark.parametrize("st", [C.CS_FD, C.CS_Q1], ids=["fd", "q1"])
@pytest.mark.parametrize("nsw", list(range(1, 10)))
@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_fused2d_jacobi_bitwise(n, st, nsw, dt):
    got, want = _run_jacobi(n, st, nsw, dt, "aligned", C.CS_PASS_AUTO, 2000 + nsw)
    assert np.array_equal(got, want), "max diff %g" % np.max(np.abs(got.astype(np.float64) - want))


@pytest.mark.parametrize("layout", ["compact", "odd"])
@pytest.mark.parametrize("st", [C.CS_FD, C.CS_Q1], ids=["fd", "q1"])
@pytest.mark.parametrize("mode", [C.CS_PASS_AUTO, C.CS_PASS_ONE], ids=["auto", "one"])
def test_fused2d_jacobi_layouts_and_modes(layout, st, mode):
    got, want = _run_jacobi((97, 45), st, 7, torch.float64, layout, mode, 2100)
    assert np.array_equal(got, want)
