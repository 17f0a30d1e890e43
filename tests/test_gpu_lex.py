"""Lexicographic Gauss-Seidel (hyperplane wavefronts) against the oracle's
sequential natural-order sweep: bit for bit, both stencils, 2D and 3D, FP64
and FP32, grids with ragged extents and a random Dirichlet halo."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_04033_amd import colsten as C

import gpu_util as G

pytestmark = pytest.mark.gpu

NP = {torch.float64: np.float64, torch.float32: np.float32}
CASES = [(2, (1, 1)), (2, (37, 21)), (3, (1, 2, 3)), (3, (17, 9, 12)), (3, (33, 5, 7))]


@pytest.mark.parametrize("dim,n", CASES, ids=lambda p: "x".join(map(str, p)) if isinstance(p, tuple) else str(p))
@pytest.mark.parametrize("st", [C.CS_FD, C.CS_Q1], ids=["fd", "q1"])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_lex_sweeps_bitwise(dim, n, st, dt):
    u, b = G.case(dim, n, seed=970 + dim)
    h = 1.0 / (max(n) + 1)
    ref, bo = u.astype(NP[dt]), b.astype(NP[dt])
    O.lex_sweeps(ref, bo, 2, dim=dim, stencil=st, h=h)
    ug, bg = G.upload(u, dt), G.upload(b, dt)
    g = C.Grid(ug, bg, dim=dim, stencil=st, h=h)
    g.gs_lex(2)
    torch.cuda.synchronize()
    assert np.array_equal(ug.detach().cpu().numpy(), ref)


def test_lex_differs_from_coloured():
    u, b = G.case(3, (9, 8, 7), seed=980)
    ug, bg = G.upload(u), G.upload(b)
    uc = G.upload(u)
    C.Grid(ug, bg, dim=3, stencil=C.CS_FD, h=0.1).gs_lex(1)
    C.Grid(uc, bg, dim=3, stencil=C.CS_FD, h=0.1).gs(1)
    torch.cuda.synchronize()
    assert not torch.equal(ug, uc)
