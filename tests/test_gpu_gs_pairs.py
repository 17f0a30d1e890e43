"""Fused red-black sweeps run two per pass over memory (3D, 7-point): the
second sweep trails the first by two planes inside one pass.  Even and odd
sweep counts (paired passes, plus one single pass for an odd count) must give
the oracle's coloured iterate bit for bit, on grids of several tiles and
z-chunks with ragged tails, every layout, both colour parities, a random
Dirichlet halo, FP64 and FP32."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_04033_amd import colsten as C

import gpu_util as G

pytestmark = pytest.mark.gpu

NP = {torch.float64: np.float64, torch.float32: np.float32}
SHAPES = [(1, 1, 1), (2, 3, 4), (5, 7, 3), (33, 9, 20), (65, 34, 7), (130, 20, 11), (64, 16, 70),
          (70, 18, 40)]


@pytest.mark.parametrize("n", SHAPES, ids=lambda p: "x".join(map(str, p)))
@pytest.mark.parametrize("nsw", [1, 2, 4, 5])
@pytest.mark.parametrize("mode", [C.CS_PASS_TWO, C.CS_PASS_ONE], ids=["two", "one"])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("layout", ["aligned", "compact", "odd"])
@pytest.mark.parametrize("parity", [0, 1])
def test_paired_fused_gs_bitwise(n, nsw, mode, dt, layout, parity):
    u, b = G.case(3, n, seed=1600 + nsw + 10 * parity)
    h = 1.0 / (max(n) + 1)
    uo, bo = u.astype(NP[dt]), b.astype(NP[dt])
    O.gs_sweeps(uo, bo, nsw, dim=3, stencil=O.FD, h=h, parity=parity)
    ug, bg = G.upload(u, dt, layout=layout), G.upload(b, dt, layout=layout)
    g = C.Grid(ug, bg, dim=3, stencil=C.CS_FD, h=h, parity=parity)
    g.set_pass_mode(mode)
    g.gs(nsw, tmp=C.grid_like(ug))
    torch.cuda.synchronize()
    got = ug.detach().cpu().numpy()
    assert np.array_equal(got, uo), "max diff %g" % np.max(np.abs(got.astype(np.float64) - uo))


@pytest.mark.parametrize("n", SHAPES, ids=lambda p: "x".join(map(str, p)))
@pytest.mark.parametrize("nsw", [2, 5])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("layout", ["aligned", "odd"])
@pytest.mark.parametrize("parity", [0, 1])
def test_paired_fused_q1_gs_bitwise(n, nsw, dt, layout, parity):
    """Two 8-colour 27-point sweeps per pass (the second trailing the first
    by two planes, rings of 7 and 3 points recomputed per tile): the oracle's
    coloured iterate bit for bit, with an odd count's last sweep alone."""
    u, b = G.case(3, n, seed=1650 + nsw + 10 * parity)
    h = 1.0 / (max(n) + 1)
    uo, bo = u.astype(NP[dt]), b.astype(NP[dt])
    O.gs_sweeps(uo, bo, nsw, dim=3, stencil=O.Q1, h=h, parity=parity)
    ug, bg = G.upload(u, dt, layout=layout), G.upload(b, dt, layout=layout)
    g = C.Grid(ug, bg, dim=3, stencil=C.CS_Q1, h=h, parity=parity)
    g.set_pass_mode(C.CS_PASS_TWO)
    assert g.sweeps_per_pass() == 2
    g.gs(nsw, tmp=C.grid_like(ug))
    torch.cuda.synchronize()
    got = ug.detach().cpu().numpy()
    assert np.array_equal(got, uo), "max diff %g" % np.max(np.abs(got.astype(np.float64) - uo))


def test_paired_fused_q1_gs_256_full_size():
    """The 27-point double sweep at 256^3 (several tiles and z-chunks), four
    sweeps from the seeded uniform RHS, bit for bit against the oracle."""
    from paper_1810_04033_amd import inputs as I
    n, h = 256, 1.0 / 257
    b = I.halo_array(I.uniform_field(2, (n, n, n)))
    u0 = I.halo_array(np.zeros((n, n, n)))
    ug, bg = G.upload(u0), G.upload(b)
    g = C.Grid(ug, bg, dim=3, stencil=C.CS_Q1, h=h)
    g.set_pass_mode(C.CS_PASS_TWO)
    g.gs(4, tmp=C.grid_like(ug))
    O.gs_sweeps(u0, b, 4, dim=3, stencil=O.Q1, h=h)
    assert np.array_equal(G.download(ug), u0)


def test_pass_mode_choice_and_errors():
    """The automatic choice pairs the red-black sweeps on a grid that fills the
    device and not on a small one; Jacobi sweeps are paired in 3D; the 8-colour
    sweeps pair when asked to; 2D Jacobi one per pass; bad modes are rejected."""
    def grid(n, st=C.CS_FD, dim=3):
        u = C.empty_grid(n)
        return C.Grid(u, C.grid_like(u), dim=dim, stencil=st, h=0.1)

    big, small = grid((256, 256, 256)), grid((64, 64, 64))
    assert big.sweeps_per_pass() == 2 and small.sweeps_per_pass() == 1
    assert big.sweeps_per_pass(jacobi=True) == 2 and small.sweeps_per_pass(jacobi=True) == 2
    small.set_pass_mode(C.CS_PASS_TWO)
    assert small.sweeps_per_pass() == 2
    big.set_pass_mode(C.CS_PASS_ONE)
    assert big.sweeps_per_pass() == 1 and big.sweeps_per_pass(jacobi=True) == 1
    q1 = grid((256, 256, 256), st=C.CS_Q1)
    q1.set_pass_mode(C.CS_PASS_TWO)
    assert q1.sweeps_per_pass() == 2 and q1.sweeps_per_pass(jacobi=True) == 2
    two_d = grid((256, 256), dim=2)
    two_d.set_pass_mode(C.CS_PASS_ONE)
    assert two_d.sweeps_per_pass() == 1 and two_d.sweeps_per_pass(jacobi=True) == 1
    for bad in (-1, 3):
        with pytest.raises(C.ColstenError) as e:
            big.set_pass_mode(bad)
        assert e.value.status == C.CS_EINVAL
    with pytest.raises(C.ColstenError) as e:
        C.cs_sweeps_per_pass(None, False)
    assert e.value.status == C.CS_EINVAL
