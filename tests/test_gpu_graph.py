"""Captured sweep sequences (HIP graphs) against the same sweeps run eagerly.

Each graph is replayed several times with the program's own eager work and
synchronisations in between; after every replay the grid must equal the eager
run of the same total number of sweeps bit for bit (the replays continue from
the current contents of u)."""
import numpy as np
import pytest
import torch

from paper_1810_04033_amd import colsten as C
from paper_1810_04033_amd import inputs as I

import gpu_util as G

pytestmark = pytest.mark.gpu

CASES = [
    ("colour_passes_2d_fd", 2, C.CS_FD, (65, 33), False, False),
    ("colour_passes_3d_q1", 3, C.CS_Q1, (17, 9, 12), False, False),
    ("fused_3d_fd", 3, C.CS_FD, (33, 9, 20), True, False),
    ("fused_3d_q1", 3, C.CS_Q1, (40, 18, 11), True, False),
    ("lexicographic_3d_q1", 3, C.CS_Q1, (11, 6, 5), False, True),
]


@pytest.mark.parametrize("name,dim,st,n,use_tmp,lex", CASES, ids=[c[0] for c in CASES])
def test_graph_replays_equal_eager_sweeps(name, dim, st, n, use_tmp, lex):
    u, b = G.case(dim, n, seed=990 + dim)
    h = 1.0 / (max(n) + 1)
    ug, ue, bg = G.upload(u), G.upload(u), G.upload(b)
    tg = C.grid_like(ug) if use_tmp else None
    te = C.grid_like(ue) if use_tmp else None
    gg = C.Grid(ug, bg, dim=dim, stencil=st, h=h)
    ge = C.Grid(ue, bg, dim=dim, stencil=st, h=h)
    graph = C.Graph.of_grid(gg, 3, tmp=tg, lexicographic=lex)
    for rep in range(4):
        graph.launch()
        if lex:
            ge.gs_lex(3)
        else:
            ge.gs(3, tmp=te)
        torch.cuda.synchronize()
        assert torch.equal(ug, ue), "replay %d differs" % rep
    graph.close()


def test_batch_graph_replays_equal_eager_batch():
    edges = [(9, 7, 5), (16, 16, 16), (12, 20, 8)]
    def make():
        ps = []
        for i, e in enumerate(edges):
            shape = tuple(reversed(e))
            u = C.empty_grid(e)
            bt = C.empty_grid(e)
            u.copy_(torch.from_numpy(I.halo_array(I.uniform_field(I.stream_seed(991, i), shape))))
            bt.copy_(torch.from_numpy(I.halo_array(I.uniform_field(I.stream_seed(992, i), shape))))
            ps.append((u, bt, C.grid_like(u), C.CS_FD if i % 2 == 0 else C.CS_Q1, 1.0 / (max(e) + 1), 0))
        return ps
    pg, pe = make(), make()
    bg, be = C.Batch(pg), C.Batch(pe)
    graph = C.Graph.of_batch(bg, 2)
    for rep in range(3):
        graph.launch()
        be.gs(2)
        torch.cuda.synchronize()
        for (ua, *_), (ub, *_) in zip(pg, pe):
            assert torch.equal(ua, ub), "replay %d differs" % rep
    graph.close()
    bg.close()
    be.close()


def test_graph_arguments_rejected():
    u, b = G.case(3, (9, 8, 7), seed=993)
    ug, bg = G.upload(u), G.upload(b)
    g = C.Grid(ug, bg, dim=3, stencil=C.CS_FD, h=0.1)
    with pytest.raises(C.ColstenError) as e:
        C.Graph.of_grid(g, 0)
    assert e.value.status == C.CS_EINVAL
    with pytest.raises(C.ColstenError) as e:
        C.Graph.of_grid(g, 2, tmp=C.grid_like(ug), lexicographic=True)
    assert e.value.status == C.CS_EINVAL
    torch.cuda.synchronize()
    assert np.array_equal(ug.detach().cpu().numpy(), u)
