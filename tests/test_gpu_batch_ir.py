"""Reserved batches reassigned without allocation, and the batched refinement
steps, against their single-grid and create-time counterparts."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_04033_amd import colsten as C
from paper_1810_04033_amd import inputs as I
from paper_1810_04033_amd import solve as S

import gpu_util as G

pytestmark = pytest.mark.gpu

SHAPES = [((24, 20, 16), C.CS_FD), ((9, 30, 7), C.CS_Q1), ((40, 33, 29), C.CS_Q1),
          ((70, 18, 21), C.CS_FD), ((5, 5, 5), C.CS_Q1)]


def _ir_case(n, st, seed):
    h = 1.0 / (max(n) + 1)
    b = I.halo_array(I.uniform_field(seed, tuple(reversed(n))))
    return h, b


def test_batched_refinement_equals_single_grid_refinement():
    """Four refinement steps of five patches (both stencils, rows permuted) in
    one reserved FP32 batch give every patch's FP64 iterate and FP32
    correction bit for bit as the single-grid calls (scale rule included)."""
    rows = [7, 2, 11, 0, 5]
    cap = sum(C.residual_items(n) for n, _ in SHAPES)
    bt = C.cs_batch_reserve(8, cap)
    norms = torch.zeros(12, 3, dtype=torch.float64, device="cuda")
    scales = torch.ones(12, dtype=torch.float64, device="cuda")
    xs, bs, es, rs, ts, want = [], [], [], [], [], []
    for i, (n, st) in enumerate(SHAPES):
        h, bh = _ir_case(n, st, 40 + i)
        x = C.empty_grid(n)
        b = C.empty_grid(n)
        b.copy_(torch.from_numpy(bh))
        e = C.empty_grid(n, dtype=torch.float32)
        xs.append(x), bs.append(b), es.append(e)
        rs.append(C.empty_grid(n, dtype=torch.float32)), ts.append(C.grid_like(e))
        norms[rows[i], 1] = float(np.max(np.abs(bh)))
        # the single-grid reference: four outer steps of 7 inner sweeps
        x2, b2 = C.empty_grid(n), C.empty_grid(n)
        b2.copy_(torch.from_numpy(bh))
        e2, r2 = C.empty_grid(n, dtype=torch.float32), C.empty_grid(n, dtype=torch.float32)
        g64 = C.Grid(x2, b2, dim=3, stencil=st, h=h)
        g32 = C.Grid(e2, r2, dim=3, stencil=st, h=h)
        res = S.ir_solve(g64, g32, 0.0, inner_sweeps=7, tmp32=C.grid_like(e2), max_outer=4)
        assert res.outer == 4
        want.append((x2.cpu().numpy(), res.history))
    descs32 = [C.describe(e, dim=3, stencil=st, h=1.0 / (max(n) + 1)) for e, (n, st) in zip(es, SHAPES)]
    descs64 = [C.describe(x, dim=3, stencil=st, h=1.0 / (max(n) + 1)) for x, (n, st) in zip(xs, SHAPES)]
    C.cs_batch_assign(bt, descs32, [e.data_ptr() for e in es], [r.data_ptr() for r in rs],
                      [t.data_ptr() for t in ts], rows)
    C.cs_batch_ir_attach(bt, descs64, [x.data_ptr() for x in xs], [b.data_ptr() for b in bs])
    hist = [[] for _ in SHAPES]
    for step in range(5):
        C.cs_batch_ir_update(bt, scales.data_ptr())
        if step == 4:
            break
        C.cs_batch_ir_residual(bt, scales.data_ptr(), norms.data_ptr())
        nr = norms.cpu().numpy()
        for i in range(len(SHAPES)):
            hist[i].append(nr[rows[i], 0] / nr[rows[i], 2])
        C.cs_batch_gs_sweeps(bt, 7)
    torch.cuda.synchronize()
    for i in range(len(SHAPES)):
        x_ref, h_ref = want[i]
        assert np.array_equal(xs[i].cpu().numpy(), x_ref), SHAPES[i]
        np.testing.assert_allclose(hist[i], h_ref[:4], rtol=1e-12)
    C.cs_batch_destroy(bt)


def test_reserved_batch_reassigned_matches_created_batch():
    """A reserved batch assigned three different patch sets in a row (rows
    given, the second set smaller) sweeps and reports norms in its rows exactly
    as a batch created for each set."""
    cap = 20 * C.residual_items((64, 64, 64))
    bt = C.cs_batch_reserve(20, cap)
    norms = torch.zeros(40, 3, dtype=torch.float64, device="cuda")
    for rnd, shapes in enumerate([[(8, 8, 8), (30, 20, 10), (64, 40, 33), (17, 16, 16)],
                                  [(24, 24, 24)],
                                  [(48, 48, 48), (5, 7, 3), (16, 16, 16), (33, 9, 20), (12, 40, 20)]]):
        pa, pb = [], []
        for i, n in enumerate(shapes):
            st = (i + rnd) % 2
            u, b = G.case(3, n, seed=300 + 10 * rnd + i)
            h = 1.0 / (max(n) + 1)
            for lst in (pa, pb):
                ug, bg = G.upload(u), G.upload(b)
                lst.append((ug, bg, C.grid_like(ug), st, h, i % 2))
        rows = [39 - 3 * i - rnd for i in range(len(shapes))]
        descs = [C.describe(u, dim=3, stencil=st, h=h, parity=par) for (u, b, t, st, h, par) in pa]
        C.cs_batch_assign(bt, descs, [p[0].data_ptr() for p in pa], [p[1].data_ptr() for p in pa],
                          [p[2].data_ptr() for p in pa], rows)
        C.cs_batch_gs_sweeps(bt, 5)
        C.cs_batch_residual(bt, norms.data_ptr())
        ref = C.Batch(pb)
        ref.gs(5)
        want = ref.residual().cpu().numpy()
        got = norms.cpu().numpy()
        for i in range(len(shapes)):
            assert torch.equal(pa[i][0], pb[i][0])
            assert np.array_equal(got[rows[i]], want[i])
        ref.close()
    C.cs_batch_destroy(bt)


def test_reserved_batch_errors():
    u, b = G.case(3, (8, 8, 8), seed=5)
    ug, bg = G.upload(u), G.upload(b)
    p = (ug, bg, C.grid_like(ug))
    d = C.describe(ug, dim=3, stencil=C.CS_FD, h=1.0 / 9)
    bt = C.cs_batch_reserve(1, C.residual_items((8, 8, 8)))
    with pytest.raises(C.ColstenError):  # beyond the capacity
        C.cs_batch_assign(bt, [d, d], [ug.data_ptr()] * 2, [bg.data_ptr()] * 2, [p[2].data_ptr()] * 2)
    big = C.empty_grid((8, 64, 64))
    dbig = C.describe(big, dim=3, stencil=C.CS_FD, h=0.1)
    with pytest.raises(C.ColstenError):  # beyond the reserved partials
        C.cs_batch_assign(bt, [dbig], [big.data_ptr()], [C.grid_like(big).data_ptr()],
                          [C.grid_like(big).data_ptr()])
    with pytest.raises(C.ColstenError):  # no refinement pairing
        C.cs_batch_assign(bt, [d], [ug.data_ptr()], [bg.data_ptr()], [p[2].data_ptr()])
        sc = torch.ones(1, dtype=torch.float64, device="cuda")
        C.cs_batch_ir_update(bt, sc.data_ptr())
    with pytest.raises(C.ColstenError):  # an FP64 batch cannot be paired
        C.cs_batch_ir_attach(bt, [d], [C.grid_like(ug).data_ptr()], [bg.data_ptr()])
    C.cs_batch_destroy(bt)
    bt2 = C.cs_batch_reserve(2, 2 * C.residual_items((8, 8, 8)))
    with pytest.raises(C.ColstenError):  # two patches on one norm row
        u2, b2 = G.upload(u), G.upload(b)
        C.cs_batch_assign(bt2, [d, d], [ug.data_ptr(), u2.data_ptr()], [bg.data_ptr(), b2.data_ptr()],
                          [p[2].data_ptr(), C.grid_like(u2).data_ptr()], [3, 3])
    with pytest.raises(C.ColstenError):
        C.cs_batch_reserve(0, 1)
    C.cs_batch_destroy(bt2)
