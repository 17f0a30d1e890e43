"""Dependency-driven colour sweeps (the Hyb-depend form): tiles wait only for
their neighbour tiles' previous colour phase, with no barrier between
colours.  The same iterate as the colour passes, bit for bit, on 2D and 3D
grids of both stencils and parities, FP64 and FP32, one tile up to many tiles
per workgroup, ragged shapes; no wait gives up."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_04033_amd import colsten as C

import gpu_util as G

pytestmark = pytest.mark.gpu

NP = {torch.float64: np.float64, torch.float32: np.float32}
# 3D tiles are 32 x 16 x 8 points, 2D tiles 64 x 32: one tile, a few ragged
# tiles, and (256^2, 128 x 64 x 40, 256 x 128 x 96) up to several tiles per
# workgroup of the 256-workgroup launch
CASES = [(2, (1, 1)), (2, (5, 7)), (2, (65, 33)), (2, (256, 256)), (3, (1, 1, 1)), (3, (5, 7, 3)),
         (3, (33, 17, 9)), (3, (65, 34, 20)), (3, (128, 64, 40)), (3, (256, 128, 96))]


@pytest.mark.parametrize("dim,n", CASES, ids=lambda p: "x".join(map(str, p)) if isinstance(p, tuple) else str(p))
@pytest.mark.parametrize("st", [C.CS_FD, C.CS_Q1], ids=["fd", "q1"])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("nsw", [1, 3])
def test_dependency_sweeps_bitwise(dim, n, st, dt, nsw):
    parity = nsw % 2
    u, b = G.case(dim, n, seed=2800 + nsw)
    h = 1.0 / (max(n) + 1)
    uo, bo = u.astype(NP[dt]), b.astype(NP[dt])
    O.gs_sweeps(uo, bo, nsw, dim=dim, stencil=st, h=h, parity=parity)
    ug, bg = G.upload(u, dt, layout="odd"), G.upload(b, dt, layout="odd")
    g = C.Grid(ug, bg, dim=dim, stencil=st, h=h, parity=parity)
    g.gs_dep(nsw)
    assert g.sync_failures() == 0
    got = ug.detach().cpu().numpy()
    g.close()
    assert np.array_equal(got, uo), "max diff %g" % np.max(np.abs(got.astype(np.float64) - uo))


def test_dependency_sweeps_repeat_and_arguments():
    # the counters start from zero on every call: two calls equal one of 2 sweeps
    n = (70, 40, 20)
    u, b = G.case(3, n, seed=2900)
    h = 1.0 / 71
    uo = u.copy()
    O.gs_sweeps(uo, b, 2, dim=3, stencil=O.Q1, h=h)
    ug, bg = G.upload(u), G.upload(b)
    g = C.Grid(ug, bg, dim=3, stencil=C.CS_Q1, h=h)
    g.gs_dep(1)
    g.gs_dep(1)
    assert g.sync_failures() == 0
    assert np.array_equal(G.download(ug), uo)
    with pytest.raises(C.ColstenError) as e:
        g.gs_dep(-1)
    assert e.value.status == C.CS_EINVAL
    g.gs_dep(0)
    g.close()
