"""One GPU's z-slab of a larger grid (512 x 512 x 64, an eighth of 512^3) in
the launch configuration the slab measurement uses: the library's automatic
choice of passes and a work array, red-black and 8-colour Gauss-Seidel and
weighted Jacobi, against the oracle element by element.  Four sweeps give the
two-sweep passes where the automatic choice takes them."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_04033_amd import colsten as C

pytestmark = pytest.mark.gpu

N = (512, 512, 64)
H = 1.0 / 513
SWEEPS = 4
OMEGA = 2.0 / 3.0


@pytest.fixture(scope="module")
def rhs():
    b = C.empty_grid(N)
    C.fill_uniform(b, 2, dim=3)
    return b, np.ascontiguousarray(b.detach().cpu().numpy())


@pytest.mark.parametrize("stencil", [C.CS_FD, C.CS_Q1], ids=["fd7", "q1_27"])
@pytest.mark.parametrize("kind", ["gs", "jacobi"])
def test_slab_bitwise(rhs, stencil, kind):
    b, bh = rhs
    u = C.empty_grid(N)
    tmp = C.empty_grid(N)
    g = C.Grid(u, b, dim=3, stencil=stencil, h=H)
    ost = O.FD if stencil == C.CS_FD else O.Q1
    uo = np.zeros_like(bh)
    if kind == "gs":
        g.gs(SWEEPS, tmp=tmp)
        O.gs_sweeps(uo, bh, SWEEPS, dim=3, stencil=ost, h=H)
    else:
        g.jacobi(OMEGA, SWEEPS, tmp)
        O.jacobi_sweeps(uo, bh, SWEEPS, OMEGA, dim=3, stencil=ost, h=H)
    torch.cuda.synchronize()
    assert np.array_equal(u.detach().cpu().numpy(), uo)
    g.close()
