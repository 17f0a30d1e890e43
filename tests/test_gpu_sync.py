"""Persistent colour sweeps with a device-wide barrier between colours (the
Hyb-sync form): the same iterate as the colour passes, bit for bit, on 2D and
3D grids of both stencils and parities, FP64 and FP32, ragged shapes from one
point up; no barrier wait gives up."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_04033_amd import colsten as C

import gpu_util as G

pytestmark = pytest.mark.gpu

NP = {torch.float64: np.float64, torch.float32: np.float32}
CASES = [(2, (1, 1)), (2, (5, 7)), (2, (65, 33)), (2, (256, 256)), (3, (1, 1, 1)), (3, (5, 7, 3)),
         (3, (33, 9, 20)), (3, (65, 34, 7)), (3, (128, 64, 40))]


@pytest.mark.parametrize("dim,n", CASES, ids=lambda p: "x".join(map(str, p)) if isinstance(p, tuple) else str(p))
@pytest.mark.parametrize("st", [C.CS_FD, C.CS_Q1], ids=["fd", "q1"])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("nsw", [1, 3])
def test_persistent_sweeps_bitwise(dim, n, st, dt, nsw):
    parity = nsw % 2
    u, b = G.case(dim, n, seed=2200 + nsw)
    h = 1.0 / (max(n) + 1)
    uo, bo = u.astype(NP[dt]), b.astype(NP[dt])
    O.gs_sweeps(uo, bo, nsw, dim=dim, stencil=st, h=h, parity=parity)
    ug, bg = G.upload(u, dt), G.upload(b, dt)
    g = C.Grid(ug, bg, dim=dim, stencil=st, h=h, parity=parity)
    g.gs_sync(nsw)
    assert g.sync_failures() == 0
    got = ug.detach().cpu().numpy()
    g.close()
    assert np.array_equal(got, uo), "max diff %g" % np.max(np.abs(got.astype(np.float64) - uo))


def test_persistent_sweeps_arguments():
    u, b = G.case(3, (9, 8, 7), seed=2300)
    g = C.Grid(G.upload(u), G.upload(b), dim=3, stencil=C.CS_FD, h=0.1)
    with pytest.raises(C.ColstenError) as e:
        g.gs_sync(-1)
    assert e.value.status == C.CS_EINVAL
    g.gs_sync(0)
    assert g.sync_failures() == 0
    g.close()
