"""Schedules of small 3D grids in the automatic pass mode: up to 4096 points
every sweep runs in one workgroup with a workgroup barrier per colour, and
7-point grids of up to 1.1 M points run one launch per colour in place.  Each
must give the oracle's coloured iterate bit for bit, on both sides of the size
limits, with and without a work array, FP64 and FP32, both colour parities,
with a random Dirichlet halo."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_04033_amd import colsten as C

import gpu_util as G

pytestmark = pytest.mark.gpu

NP = {torch.float64: np.float64, torch.float32: np.float32}
# 16^3 = 4096 points (one workgroup); 17 x 16 x 16 just above; 1 point; a
# ragged shape; 7-point 100^3 and 104 x 104 x 102 around the colour-launch limit
SHAPES = [(1, 1, 1), (5, 3, 2), (16, 16, 16), (17, 16, 16), (33, 9, 20)]


@pytest.mark.parametrize("n", SHAPES, ids=lambda p: "x".join(map(str, p)))
@pytest.mark.parametrize("stencil", [C.CS_FD, C.CS_Q1], ids=["fd", "q1"])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("parity", [0, 1])
@pytest.mark.parametrize("with_tmp", [True, False], ids=["tmp", "notmp"])
def test_small_grid_schedules_bitwise(n, stencil, dt, parity, with_tmp):
    u, b = G.case(3, n, seed=3100 + parity + sum(n))
    h = 1.0 / (max(n) + 1)
    uo, bo = u.astype(NP[dt]), b.astype(NP[dt])
    O.gs_sweeps(uo, bo, 3, dim=3, stencil=stencil, h=h, parity=parity)
    ug, bg = G.upload(u, dt, layout="odd"), G.upload(b, dt, layout="odd")
    g = C.Grid(ug, bg, dim=3, stencil=stencil, h=h, parity=parity)
    g.gs(3, tmp=C.grid_like(ug) if with_tmp else None)
    torch.cuda.synchronize()
    assert np.array_equal(ug.detach().cpu().numpy(), uo)


@pytest.mark.parametrize("n", [(100, 100, 100), (104, 104, 102)], ids=lambda p: "x".join(map(str, p)))
def test_colour_launch_limit_bitwise(n):
    # 1,000,000 points run the colour launches, 1,103,232 the fused passes
    u, b = G.case(3, n, seed=3200)
    h = 1.0 / (max(n) + 1)
    uo = u.copy()
    O.gs_sweeps(uo, b, 2, dim=3, stencil=O.FD, h=h)
    ug, bg = G.upload(u), G.upload(b)
    g = C.Grid(ug, bg, dim=3, stencil=C.CS_FD, h=h)
    g.gs(2, tmp=C.grid_like(ug))
    torch.cuda.synchronize()
    assert np.array_equal(G.download(ug), uo)
