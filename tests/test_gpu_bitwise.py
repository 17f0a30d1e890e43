"""Bitwise agreement of the GPU kernels with the oracle.

Both sides add each neighbour term with one fused multiply-add in the same
lexicographic offset order and form the quotient by the centre weight as the
exact quotient rounded once, so the iterates agree bit for bit, not just within
the 1e-13 parity bound.  Checked for the fused sweeps, the colour passes and
Jacobi, both stencils, FP64 and FP32, 2D and 3D, on grids of several tiles with
ragged tails and a random Dirichlet halo."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_04033_amd import colsten as C

import gpu_util as G

pytestmark = pytest.mark.gpu

NP = {torch.float64: np.float64, torch.float32: np.float32}
CASES = [(2, (65, 33)), (3, (33, 9, 20)), (3, (65, 34, 7)), (3, (130, 20, 11))]


def _gpu(u, b, dt, dim, st, h, fn):
    ug, bg = G.upload(u, dt), G.upload(b, dt)
    g = C.Grid(ug, bg, dim=dim, stencil=st, h=h)
    fn(g, ug)
    torch.cuda.synchronize()
    return ug.detach().cpu().numpy()


@pytest.mark.parametrize("dim,n", CASES, ids=lambda p: "x".join(map(str, p)) if isinstance(p, tuple) else str(p))
@pytest.mark.parametrize("st", [C.CS_FD, C.CS_Q1], ids=["fd", "q1"])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("kind", ["fused", "passes", "jacobi"])
def test_bitwise(dim, n, st, dt, kind):
    u, b = G.case(dim, n, seed=900 + dim)
    h = 1.0 / (max(n) + 1)
    uo, bo = u.astype(NP[dt]), b.astype(NP[dt])
    if kind == "jacobi":
        O.jacobi_sweeps(uo, bo, 3, 2.0 / 3.0, dim=dim, stencil=st, h=h)
        got = _gpu(u, b, dt, dim, st, h, lambda g, ug: g.jacobi(2.0 / 3.0, 3, C.grid_like(ug)))
    else:
        O.gs_sweeps(uo, bo, 3, dim=dim, stencil=st, h=h)
        if kind == "fused":
            got = _gpu(u, b, dt, dim, st, h, lambda g, ug: g.gs(3, tmp=C.grid_like(ug)))
        else:
            got = _gpu(u, b, dt, dim, st, h, lambda g, ug: g.gs(3))
    assert got.dtype == uo.dtype
    assert np.array_equal(got, uo), "max diff %g" % np.max(np.abs(got.astype(np.float64) - uo))
