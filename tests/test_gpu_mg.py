"""Multigrid on the GPU (cs_restrict, cs_prolong_add and the V-cycle driver
above them) against the oracle's V-cycle: the transfers bit for bit on every
layout, whole V-cycles bit for bit (the sweeps and the residual are the
oracle's to the bit, so the cycle is too), FD and d-linear stencils in 2D and
3D, both colour parities; a 127^3 solve to 1e-10; and the argument checks."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_04033_amd import colsten as C
from paper_1810_04033_amd import inputs as I
from paper_1810_04033_amd import mg as MG

import gpu_util as G

pytestmark = pytest.mark.gpu

TRANSFER_SHAPES = [(3, 3), (7, 5), (65, 33), (3, 3, 3), (7, 5, 9), (33, 17, 5), (129, 9, 7)]


def _coarse(n):
    return tuple((v - 1) // 2 for v in n)


def _grid(u, b, n, stencil=C.CS_FD, h=0.01, parity=0):
    return C.Grid(u, b, dim=len(n), stencil=stencil, h=h, parity=parity)


@pytest.mark.parametrize("n", TRANSFER_SHAPES, ids=lambda p: "x".join(map(str, p)))
@pytest.mark.parametrize("layout", ["aligned", "compact", "odd"])
def test_restriction_bitwise(n, layout):
    dim = len(n)
    r, _ = G.case(dim, n, seed=2100 + sum(n))
    uc0, bc0 = G.case(dim, _coarse(n), seed=2200 + sum(n))
    bo, uo = bc0.copy(), uc0.copy()
    O.restrict(r, bo, uo, dim=dim)
    rg = G.upload(r, layout=layout)
    ufg, bfg = G.upload(np.zeros_like(r), layout=layout), G.upload(np.zeros_like(r), layout=layout)
    ucg, bcg = G.upload(uc0, layout=layout), G.upload(bc0, layout=layout)
    gf, gc = _grid(ufg, bfg, n), _grid(ucg, bcg, _coarse(n))
    C.restrict(gf, rg, gc)
    torch.cuda.synchronize()
    assert np.array_equal(G.download(bcg), bo)
    assert np.array_equal(G.download(ucg), uo)  # interior zeroed, halo kept


@pytest.mark.parametrize("n", TRANSFER_SHAPES, ids=lambda p: "x".join(map(str, p)))
@pytest.mark.parametrize("layout", ["aligned", "compact", "odd"])
def test_interpolation_bitwise(n, layout):
    dim = len(n)
    uf, bf = G.case(dim, n, seed=2300 + sum(n))
    uc, bc = G.case(dim, _coarse(n), seed=2400 + sum(n))  # random coarse halo too
    want = uf.copy()
    O.prolong_add(uc, want, dim=dim)
    ufg, bfg = G.upload(uf, layout=layout), G.upload(bf, layout=layout)
    ucg, bcg = G.upload(uc, layout=layout), G.upload(bc, layout=layout)
    C.prolong_add(_grid(ucg, bcg, _coarse(n)), _grid(ufg, bfg, n))
    torch.cuda.synchronize()
    assert np.array_equal(G.download(ufg), want)


@pytest.mark.parametrize("n,stencil", [((31, 31, 31), C.CS_FD), ((31, 31, 31), C.CS_Q1),
                                       ((15, 7, 31), C.CS_FD), ((63, 63), C.CS_FD),
                                       ((63, 127), C.CS_Q1), ((64, 33, 17), C.CS_Q1)],
                         ids=lambda p: "x".join(map(str, p)) if isinstance(p, tuple) else str(p))
@pytest.mark.parametrize("parity", [0, 1])
def test_vcycles_bitwise(n, stencil, parity):
    dim = len(n)
    h = 1.0 / (max(n) + 1)
    _, b = G.case(dim, n, seed=2500 + parity)
    uo = np.zeros_like(b)
    for _ in range(3):
        O.mg_vcycle(uo, b, dim=dim, stencil=stencil, h=h, parity=parity)
    ug, bg = G.upload(np.zeros_like(b)), G.upload(b)
    g = C.Grid(ug, bg, dim=dim, stencil=stencil, h=h, parity=parity)
    mg = MG.Multigrid(g)
    assert mg.depth == (1 if not O.mg_coarsens(n) else
                        1 + min(int(np.log2(v + 1)) for v in n) - 1)
    for _ in range(3):
        mg.cycle()
    torch.cuda.synchronize()
    assert np.array_equal(G.download(ug), uo)


@pytest.mark.parametrize("stencil", [C.CS_FD, C.CS_Q1])
def test_solve_127_to_1e10(stencil):
    n = (127, 127, 127)
    h = 1.0 / 128
    b = C.empty_grid(n)
    C.fill_uniform(b, 7, dim=3)
    u = C.empty_grid(n)
    g = C.Grid(u, b, dim=3, stencil=stencil, h=h)
    res = MG.Multigrid(g).solve(1e-10, max_cycles=30)
    assert res.converged and res.rel_residual <= 1e-10
    assert res.outer <= (12 if stencil == C.CS_FD else 8)
    # per-cycle factors well below one throughout (h-independent convergence)
    f = [res.history[i + 1] / res.history[i] for i in range(1, len(res.history) - 1)]
    assert max(f) <= (0.12 if stencil == C.CS_FD else 0.03)


def test_fp32_cycles_converge():
    n = (63, 63, 63)
    b = C.empty_grid(n, dtype=torch.float32)
    C.fill_uniform(b, 9, dim=3)
    u = C.empty_grid(n, dtype=torch.float32)
    g = C.Grid(u, b, dim=3, stencil=C.CS_FD, h=1.0 / 64)
    res = MG.Multigrid(g).solve(1e-5, max_cycles=20)
    assert res.converged and res.outer <= 6


def test_argument_checks():
    f_u, f_b = C.empty_grid((7, 7, 7)), C.empty_grid((7, 7, 7))
    r = C.grid_like(f_u)
    gf = C.Grid(f_u, f_b, dim=3, stencil=C.CS_FD, h=0.125)
    bad_u, bad_b = C.empty_grid((4, 3, 3)), C.empty_grid((4, 3, 3))
    gbad = C.Grid(bad_u, bad_b, dim=3, stencil=C.CS_FD, h=0.25)
    with pytest.raises(C.ColstenError):
        C.restrict(gf, r, gbad)
    with pytest.raises(C.ColstenError):
        C.prolong_add(gbad, gf)
    c_u, c_b = C.empty_grid((3, 3, 3)), C.empty_grid((3, 3, 3))
    gq = C.Grid(c_u, c_b, dim=3, stencil=C.CS_Q1, h=0.25)
    with pytest.raises(C.ColstenError):  # stencils differ
        C.restrict(gf, r, gq)
    gc = C.Grid(c_u, c_b, dim=3, stencil=C.CS_FD, h=0.25)
    with pytest.raises(C.ColstenError):  # r is the fine iterate
        C.restrict(gf, f_u, gc)
    C.restrict(gf, r, gc)
    C.prolong_add(gc, gf)
    with pytest.raises(C.ColstenError):  # residual with neither r nor norms
        C.cs_residual(gf.handle, 0, 0)
    torch.cuda.synchronize()


def test_residual_array_without_norms_bitwise():
    n = (33, 17, 9)
    u, b = G.case(3, n, seed=2600)
    h = 1.0 / 34
    _, want = O.residual(u, b, dim=3, stencil=O.FD, h=h, want_r=True)
    ug, bg = G.upload(u), G.upload(b)
    g = C.Grid(ug, bg, dim=3, stencil=C.CS_FD, h=h)
    r = C.grid_like(ug)
    assert g.residual(r=r, want_norms=False) is None
    torch.cuda.synchronize()
    assert np.array_equal(O.interior(G.download(r)), O.interior(want))


@pytest.mark.parametrize("n,stencil", [((31, 31, 31), C.CS_FD), ((15, 15, 15), C.CS_Q1),
                                       ((63, 31), C.CS_FD)],
                         ids=lambda p: "x".join(map(str, p)) if isinstance(p, tuple) else str(p))
def test_vcycle_graph_replays_bitwise(n, stencil):
    # a captured cycle, replayed several times with eager work and host
    # synchronisation between the replays, equals the eager cycles every time
    dim = len(n)
    h = 1.0 / (max(n) + 1)
    _, b = G.case(dim, n, seed=2700)
    ua, ba = G.upload(np.zeros_like(b)), G.upload(b)
    ub, bb = G.upload(np.zeros_like(b)), G.upload(b)
    mga = MG.Multigrid(C.Grid(ua, ba, dim=dim, stencil=stencil, h=h))
    mgb = MG.Multigrid(C.Grid(ub, bb, dim=dim, stencil=stencil, h=h))
    mgb.capture()
    uo = np.zeros_like(b)
    for _ in range(4):
        mga.cycle()
        mgb.cycle_graph()
        O.mg_vcycle(uo, b, dim=dim, stencil=stencil, h=h)
        torch.cuda.synchronize()
        junk = torch.ones(1 << 16, device="cuda", dtype=torch.float64)
        assert float((junk * 2).sum()) == 2.0 * (1 << 16)
        assert np.array_equal(G.download(ub), G.download(ua))
        assert np.array_equal(G.download(ub), uo)
    res = mgb.solve(1e-10, max_cycles=30, graph=True)
    assert res.converged
    mgb.close()


def test_graph_end_needs_a_capturing_stream():
    h = ctypes.c_void_p()
    s = torch.cuda.current_stream().cuda_stream
    assert C.lib().cs_graph_end(ctypes.c_void_p(s), ctypes.byref(h)) == C.CS_EINVAL
    assert C.lib().cs_graph_end(None, ctypes.byref(h)) == C.CS_EINVAL


@pytest.mark.parametrize("stencil", [C.CS_FD, C.CS_Q1], ids=["fd7", "q1_27"])
def test_vcycle_255_bitwise(stencil):
    # the multigrid workload's size and launch configuration: one V(2,2)-cycle
    # from u = 0 on 255^3 with the device-made right-hand side, against the
    # oracle's cycle element by element
    n = (255, 255, 255)
    h = 1.0 / 256
    b = C.empty_grid(n)
    C.fill_uniform(b, 2, dim=3)
    u = C.empty_grid(n)
    mg = MG.Multigrid(C.Grid(u, b, dim=3, stencil=stencil, h=h))
    mg.cycle()
    torch.cuda.synchronize()
    bh = np.ascontiguousarray(b.detach().cpu().numpy())
    uo = np.zeros_like(bh)
    O.mg_vcycle(uo, bh, dim=3, stencil=O.FD if stencil == C.CS_FD else O.Q1, h=h)
    assert np.array_equal(u.detach().cpu().numpy(), uo)
    mg.close()


@pytest.mark.parametrize("stencil", [C.CS_FD, C.CS_Q1], ids=["fd7", "q1_27"])
def test_fp32_cycles_inside_fp64_refinement(stencil):
    # FP32 V-cycles as the inner solve of FP64 iterative refinement reach an
    # FP64 tolerance FP32 alone cannot, in a few refinement steps; the final
    # residual is recomputed by the oracle
    from paper_1810_04033_amd import solve as S
    n = (63, 63, 63)
    h = 1.0 / 64
    b = C.empty_grid(n)
    C.fill_uniform(b, 11, dim=3)
    u = C.empty_grid(n)
    g64 = C.Grid(u, b, dim=3, stencil=stencil, h=h)
    e = C.empty_grid(n, dtype=torch.float32)
    r32 = C.empty_grid(n, dtype=torch.float32)
    g32 = C.Grid(e, r32, dim=3, stencil=stencil, h=h)
    mg32 = MG.Multigrid(g32)

    def inner(s):
        for _ in range(3):
            mg32.cycle(stream=s)

    res = S.ir_solve(g64, g32, 1e-10, inner_sweeps=3, inner=inner, max_outer=10)
    torch.cuda.synchronize()
    assert res.converged and res.outer <= 4
    nr = O.residual(u.detach().cpu().numpy(), b.detach().cpu().numpy(), dim=3,
                    stencil=O.FD if stencil == C.CS_FD else O.Q1, h=h)
    assert nr[0] / nr[2] <= 1e-10
    mg32.close()
