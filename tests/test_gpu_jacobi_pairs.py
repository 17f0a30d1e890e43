"""Jacobi sweeps run two per pass over memory (3D, both stencils): the
intermediate iterate is computed on the tile grown by one point and kept on chip.  Even and
odd sweep counts (paired passes, plus one single pass for an odd count) must
give the oracle's iterate bit for bit, on grids of several tiles and z-chunks
with ragged tails, every layout, a random Dirichlet halo, FP64 and FP32."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_04033_amd import colsten as C

import gpu_util as G

pytestmark = pytest.mark.gpu

NP = {torch.float64: np.float64, torch.float32: np.float32}
SHAPES = [(1, 1, 1), (2, 3, 4), (5, 7, 3), (33, 9, 20), (65, 34, 7), (130, 20, 11), (64, 8, 40)]


@pytest.mark.parametrize("n", SHAPES, ids=lambda p: "x".join(map(str, p)))
@pytest.mark.parametrize("nsw", [1, 2, 4, 5])
@pytest.mark.parametrize("mode", [C.CS_PASS_TWO, C.CS_PASS_ONE], ids=["two", "one"])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("layout", ["aligned", "compact", "odd"])
@pytest.mark.parametrize("st", [C.CS_FD, C.CS_Q1], ids=["fd", "q1"])
def test_paired_jacobi_bitwise(n, nsw, mode, dt, layout, st):
    u, b = G.case(3, n, seed=1500 + nsw)
    h = 1.0 / (max(n) + 1)
    omega = 0.8
    uo, bo = u.astype(NP[dt]), b.astype(NP[dt])
    O.jacobi_sweeps(uo, bo, nsw, omega, dim=3, stencil=st, h=h)
    ug, bg = G.upload(u, dt, layout=layout), G.upload(b, dt, layout=layout)
    g = C.Grid(ug, bg, dim=3, stencil=st, h=h)
    g.set_pass_mode(mode)
    g.jacobi(omega, nsw, C.grid_like(ug))
    torch.cuda.synchronize()
    got = ug.detach().cpu().numpy()
    assert np.array_equal(got, uo), "max diff %g" % np.max(np.abs(got.astype(np.float64) - uo))
