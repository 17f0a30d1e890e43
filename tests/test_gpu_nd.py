"""Gauss-Seidel in the nested-dissection ordering on the GPU (one launch per
tree height, one thread per node) against the oracle's recursive sweep: bit
for bit in FP64 on 2D and 3D grids of both stencils, several leaf sizes
(several tree levels), ragged shapes and a random Dirichlet halo; FP32 within
its rounding; the tree rebuilt when the leaf size changes."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_04033_amd import colsten as C

import gpu_util as G

pytestmark = pytest.mark.gpu

CASES = [((1, 1, 1), 1), ((20, 13), 4), ((64, 64), 16), ((9, 7, 10), 3), ((33, 17, 20), 8),
         ((40, 40, 40), 16), ((65, 34, 7), 5)]


@pytest.mark.parametrize("n,leaf", CASES, ids=lambda p: "x".join(map(str, p)) if isinstance(p, tuple) else str(p))
@pytest.mark.parametrize("st", [C.CS_FD, C.CS_Q1], ids=["fd", "q1"])
@pytest.mark.parametrize("nsw", [1, 2])
def test_nd_sweeps_bitwise(n, leaf, st, nsw):
    dim = len(n)
    u, b = G.case(dim, n, seed=3300 + nsw)
    h = 1.0 / (max(n) + 1)
    uo = u.copy()
    O.nd_sweeps(uo, b, nsw, dim=dim, stencil=st, h=h, leaf=leaf)
    ug, bg = G.upload(u, layout="odd"), G.upload(b, layout="odd")
    g = C.Grid(ug, bg, dim=dim, stencil=st, h=h)
    g.gs_nd(nsw, leaf=leaf)
    torch.cuda.synchronize()
    got = G.download(ug)
    g.close()
    assert np.array_equal(got, uo), "max diff %g" % np.max(np.abs(got - uo))


def test_nd_fp32_and_leaf_change():
    n = (30, 21, 17)
    u, b = G.case(3, n, seed=3400)
    h = 1.0 / 31
    uo = u.copy()
    O.nd_sweeps(uo, b, 1, dim=3, stencil=O.Q1, h=h, leaf=4)
    O.nd_sweeps(uo, b, 1, dim=3, stencil=O.Q1, h=h, leaf=7)
    ug, bg = G.upload(u), G.upload(b)
    g = C.Grid(ug, bg, dim=3, stencil=C.CS_Q1, h=h)
    g.gs_nd(1, leaf=4)
    g.gs_nd(1, leaf=7)  # another tree
    torch.cuda.synchronize()
    assert np.array_equal(G.download(ug), uo)
    u32, b32 = G.upload(u, torch.float32), G.upload(b, torch.float32)
    g32 = C.Grid(u32, b32, dim=3, stencil=C.CS_Q1, h=h)
    g32.gs_nd(1, leaf=4)
    g32.gs_nd(1, leaf=7)
    torch.cuda.synchronize()
    assert G.relmax(G.download(u32), uo) <= 1e-5
    with pytest.raises(C.ColstenError) as e:
        g.gs_nd(1, leaf=0)
    assert e.value.status == C.CS_EINVAL
    g.close()
    g32.close()
