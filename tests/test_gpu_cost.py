"""GPU sweeps with the expensive stencil evaluation S(k) against the oracle.

cs_gs_sweeps_cost must give the oracle's S(k) iterate (and hence the k = 0
iterate) bit for bit, for fixed and mesh-varying k, both stencils, 2D and 3D,
FP64 and FP32; invalid cost arguments are rejected before any launch."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_04033_amd import colsten as C

import gpu_util as G

pytestmark = pytest.mark.gpu

NP = {torch.float64: np.float64, torch.float32: np.float32}
CASES = [(2, (65, 33)), (2, (130, 7)), (3, (33, 9, 20)), (3, (65, 14, 5))]


@pytest.mark.parametrize("dim,n", CASES, ids=lambda p: "x".join(map(str, p)) if isinstance(p, tuple) else str(p))
@pytest.mark.parametrize("st", [C.CS_FD, C.CS_Q1], ids=["fd", "q1"])
@pytest.mark.parametrize("kmax,hetero", [(0, 0), (5, 0), (40, 1)])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_cost_sweeps_bitwise(dim, n, st, kmax, hetero, dt):
    u, b = G.case(dim, n, seed=950 + dim)
    h = 1.0 / (max(n) + 1)
    if dt == torch.float64:
        ref = u.copy()
        O.gs_sweeps_cost(ref, b, 2, kmax, hetero, dim=dim, stencil=st, h=h)
    else:
        ref = u.astype(np.float32)
        O.gs_sweeps(ref, b.astype(np.float32), 2, dim=dim, stencil=st, h=h)
    ug, bg = G.upload(u, dt), G.upload(b, dt)
    g = C.Grid(ug, bg, dim=dim, stencil=st, h=h)
    g.gs_cost(2, kmax, hetero=bool(hetero))
    torch.cuda.synchronize()
    got = ug.detach().cpu().numpy()
    assert np.array_equal(got, ref)


def test_cost_arguments_rejected():
    u, b = G.case(3, (9, 8, 7), seed=960)
    ug, bg = G.upload(u), G.upload(b)
    g = C.Grid(ug, bg, dim=3, stencil=C.CS_Q1, h=0.1)
    for args in [(1, -1, 0), (1, 100001, 0), (1, 5, 2), (-1, 5, 0)]:
        with pytest.raises(C.ColstenError) as e:
            C.cs_gs_sweeps_cost(g.handle, *args)
        assert e.value.status == C.CS_EINVAL
    torch.cuda.synchronize()
    assert np.array_equal(ug.detach().cpu().numpy(), u)
