"""Batched patches: every patch of a batch against the oracle, the same patch
alone and in a mix (bitwise), and the full 4096-patch workload on samples."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_04033_amd import colsten as C
from paper_1810_04033_amd import inputs as I

import gpu_util as G

pytestmark = pytest.mark.gpu

NP = {torch.float64: np.float64, torch.float32: np.float32}
TOL = {torch.float64: 1e-13, torch.float32: 1e-6}


def _patch(n, st, dt, parity, seed, layout="aligned"):
    u, b = G.case(3, n, seed)
    h = 1.0 / (max(n) + 1)
    ug, bg = G.upload(u, dt, layout), G.upload(b, dt, layout)
    return dict(n=n, st=st, dt=dt, parity=parity, h=h, u0=u, b=b, ug=ug, bg=bg, tmp=C.grid_like(ug))


def _batch(ps):
    return C.Batch([(p["ug"], p["bg"], p["tmp"], p["st"], p["h"], p["parity"]) for p in ps])


def _oracle(p, nsw):
    uo, bo = p["u0"].astype(NP[p["dt"]]), p["b"].astype(NP[p["dt"]])
    O.gs_sweeps(uo, bo, nsw, dim=3, stencil=p["st"], h=p["h"], parity=p["parity"])
    return uo.astype(np.float64)


SHAPES = [(1, 1, 1), (2, 3, 4), (5, 7, 3), (8, 8, 8), (16, 16, 16), (17, 9, 12), (24, 24, 24),
          (33, 20, 18), (48, 48, 48), (64, 64, 64), (70, 13, 65), (40, 66, 9)]


def _set_policies(tile=(0, 0), resident=3, colour=-1):
    """Batch policies of every stencil and dtype (the defaults restore them)."""
    for st in (C.CS_FD, C.CS_Q1):
        for dt in (C.CS_F64, C.CS_F32):
            C.cs_batch_tile_policy(st, dt, *tile)
            C.cs_batch_resident_policy(st, dt, resident)
            C.cs_batch_colour_policy(st, dt, colour)


@pytest.fixture
def tiles_only_for_small_groups():
    """Small groups keep the tile kernels (colour passes off) during a test."""
    _set_policies(colour=0)
    yield
    _set_policies()


@pytest.mark.parametrize("policy", ["default", "all_tile_classes", "colour_passes"])
@pytest.mark.parametrize("nsw", [1, 2, 3, 4, 5])
def test_mixed_batch_matches_oracle(nsw, policy):
    """A mixed batch (both stencils, FP64 and FP32, shapes from 1^3 to 70 x 13 x
    65, both parities, odd layouts) equals the oracle: under the default
    policies (this small batch's tiled groups go to the colour passes), with
    every tile class in use (small and middle tiles for the smaller patches,
    nothing resident, no colour passes), and with every patch on the colour
    passes."""
    if policy == "all_tile_classes":
        _set_policies((16, 40), 0, 0)
    elif policy == "colour_passes":
        _set_policies(resident=0, colour=1 << 40)
    try:
        _mixed_batch_case(nsw)
    finally:
        _set_policies()


def _mixed_batch_case(nsw):
    ps = []
    for i, n in enumerate(SHAPES):
        for st in (C.CS_FD, C.CS_Q1):
            dt = torch.float64 if (i + st) % 3 else torch.float32
            ps.append(_patch(n, st, dt, (i // 2) % 2, seed=1000 + 7 * i + st,
                             layout="odd" if i % 4 == 3 else "aligned"))
    bt = _batch(ps)
    bt.gs(nsw)
    norms = bt.residual().cpu().numpy()
    torch.cuda.synchronize()
    for i, p in enumerate(ps):
        ref = _oracle(p, nsw)
        got = G.download(p["ug"])
        assert G.relmax(got, ref) <= TOL[p["dt"]], (p["n"], p["st"], p["dt"])
        want = O.residual(ref.astype(NP[p["dt"]]), p["b"].astype(NP[p["dt"]]), dim=3,
                          stencil=p["st"], h=p["h"])
        np.testing.assert_allclose(norms[i], want, rtol=1e-11 if p["dt"] == torch.float64 else 1e-5)


def test_patch_alone_equals_patch_in_mix():
    mix = [_patch(n, st, torch.float64, 0, seed=2000 + 3 * i + st)
           for i, n in enumerate(SHAPES) for st in (C.CS_FD, C.CS_Q1)]
    probe = [_patch((33, 20, 18), C.CS_Q1, torch.float64, 0, seed=77),
             _patch((24, 24, 24), C.CS_FD, torch.float64, 1, seed=78)]
    alone = [_patch(p["n"], p["st"], p["dt"], p["parity"], seed=s) for p, s in zip(probe, (77, 78))]
    bt_mix = _batch(mix[:5] + probe[:1] + mix[5:] + probe[1:])
    bt_mix.gs(5)
    n_mix = bt_mix.residual().cpu().numpy()
    for j, p in enumerate(alone):
        ba = _batch([p])
        ba.gs(5)
        n_alone = ba.residual().cpu().numpy()
        torch.cuda.synchronize()
        assert torch.equal(p["ug"], probe[j]["ug"])
        row = 5 if j == 0 else len(mix) + 1
        assert np.array_equal(n_alone[0], n_mix[row])


def test_batch_equals_single_grid_fused_path():
    p = _patch((40, 33, 29), C.CS_Q1, torch.float64, 1, seed=90)
    q = _patch((40, 33, 29), C.CS_Q1, torch.float64, 1, seed=90)
    bt = _batch([p])
    bt.gs(6)
    g = C.Grid(q["ug"], q["bg"], dim=3, stencil=C.CS_Q1, h=q["h"], parity=1)
    g.gs(6, tmp=q["tmp"])
    torch.cuda.synchronize()
    assert torch.equal(p["ug"], q["ug"])


def test_bad_batches_are_rejected():
    p = _patch((8, 8, 8), C.CS_FD, torch.float64, 0, seed=5)
    with pytest.raises(C.ColstenError):
        C.Batch([(p["ug"], p["bg"], p["ug"], C.CS_FD, p["h"], 0)])
    d = C.describe(p["ug"], dim=3, stencil=C.CS_FD, h=p["h"])
    d.n[2] = 100000
    with pytest.raises(C.ColstenError):
        C.cs_batch_create([d], [p["ug"].data_ptr()], [p["bg"].data_ptr()], [p["tmp"].data_ptr()])
    with pytest.raises(C.ColstenError):
        C.cs_batch_create([], [], [], [])


def test_patch_workload_4096_sampled():
    """4096 cubic patches, edges uniform over {8,16,24,32,48,64}, zero halo,
    seeded uniform RHS (stream = patch id), u0 = 0, 20 red-black sweeps in one
    batch; sampled patches compared with the oracle element by element, every
    patch's norms checked against the initial ones."""
    edges = I.patch_edges(3, 4096)
    ps = []
    for i, e in enumerate(edges):
        u = C.empty_grid((e, e, e))
        b = C.empty_grid((e, e, e))
        bh = I.halo_array(I.uniform_field(I.stream_seed(3, i), (e, e, e)))
        b.copy_(torch.from_numpy(bh))
        ps.append((u, b, C.grid_like(u), C.CS_FD, 1.0 / (e + 1), 0))
    bt = C.Batch(ps)
    n0 = bt.residual().clone()
    bt.gs(20)
    n1 = bt.residual()
    torch.cuda.synchronize()
    n0, n1 = n0.cpu().numpy(), n1.cpu().numpy()
    assert np.all(np.isfinite(n1)) and np.all(n1[:, 0] < n0[:, 0])
    seen = {}
    for i, e in enumerate(edges):
        if seen.get(e, 0) >= (1 if e == 64 else 2):
            continue
        seen[e] = seen.get(e, 0) + 1
        bh = I.halo_array(I.uniform_field(I.stream_seed(3, i), (e, e, e)))
        uo = I.halo_array(np.zeros((e, e, e)))
        O.gs_sweeps(uo, bh, 20, dim=3, stencil=O.FD, h=1.0 / (e + 1))
        assert G.relmax(G.download(ps[i][0]), uo) <= 1e-13
        np.testing.assert_allclose(n1[i], O.residual(uo, bh, dim=3, stencil=O.FD, h=1.0 / (e + 1)),
                                   rtol=1e-11)


def test_sweeps_per_pass_by_tile_class(tiles_only_for_small_groups):
    """Patches of the large 7-point tile class run two sweeps per pass, the
    other tiled ones (27-point here) one, patches that fit in LDS all sweeps of
    a call in one pass (reported as 0), and patches streamed through one
    workgroup up to three per pass; bad queries are rejected."""
    ps = [_patch(n, st, torch.float64, 0, seed=1700 + i)
          for i, (n, st) in enumerate([((8, 8, 8), C.CS_FD), ((64, 64, 64), C.CS_FD),
                                       ((64, 64, 64), C.CS_Q1), ((30, 30, 30), C.CS_FD)])]
    bt = _batch(ps)
    # one streamable 7-point patch is too few to stream by default: it takes
    # the large tiles, two sweeps per pass
    assert [bt.sweeps_per_pass(i) for i in range(4)] == [0, 2, 1, 2]
    for bad in (-1, 4):
        with pytest.raises(C.ColstenError) as e:
            bt.sweeps_per_pass(bad)
        assert e.value.status == C.CS_EINVAL
    bt.close()
    C.cs_batch_resident_policy(C.CS_FD, C.CS_F64, 7)
    try:
        bt = _batch(ps)
        assert [bt.sweeps_per_pass(i) for i in range(4)] == [0, 2, 1, 3]
        bt.close()
    finally:
        C.cs_batch_resident_policy(C.CS_FD, C.CS_F64, 3)
    # by default these small tiled groups take the colour passes
    _set_policies()
    bt = _batch(ps)
    assert [bt.sweeps_per_pass(i) for i in range(4)] == [0, 1, 1, 1]
    bt.close()


def test_pass_policy_one_sweep_per_pass_same_iterate(tiles_only_for_small_groups):
    """With the pass policy off, the large 7-point class runs one sweep per
    pass and gives the same iterate bit for bit; bad policies are rejected."""
    shapes = [(64, 64, 64), (48, 50, 40), (8, 8, 8)]
    res = {}
    for pair in (1, 0):
        C.cs_batch_pass_policy(C.CS_FD, C.CS_F64, pair)
        C.cs_batch_resident_policy(C.CS_FD, C.CS_F64, 1)  # no plane streaming: tiles only
        try:
            ps = [_patch(n, C.CS_FD, torch.float64, i % 2, seed=1800 + i) for i, n in enumerate(shapes)]
            bt = _batch(ps)
            per = [bt.sweeps_per_pass(i) for i in range(len(ps))]
            bt.gs(5)
            torch.cuda.synchronize()
            res[pair] = ([G.download(p["ug"]) for p in ps], per)
            bt.close()
        finally:
            C.cs_batch_pass_policy(C.CS_FD, C.CS_F64, 1)
            C.cs_batch_resident_policy(C.CS_FD, C.CS_F64, 3)
    assert res[1][1] == [2, 2, 0] and res[0][1] == [1, 1, 0]
    for a, b in zip(res[1][0], res[0][0]):
        assert np.array_equal(a, b)
    for bad in ((2, 0, 1), (0, 2, 1), (0, 0, 2)):
        with pytest.raises(C.ColstenError) as e:
            C.cs_batch_pass_policy(*bad)
        assert e.value.status == C.CS_EINVAL


RESIDENT = [((1, 1, 1), torch.float64, 1), ((2, 3, 4), torch.float64, 1), ((8, 8, 8), torch.float64, 1),
            ((16, 16, 16), torch.float64, 1), ((17, 16, 16), torch.float64, 2),
            ((24, 24, 24), torch.float64, 2), ((25, 24, 24), torch.float64, 0),
            ((12, 40, 20), torch.float64, 2), ((7, 5, 61), torch.float64, 2),
            ((16, 16, 16), torch.float32, 1), ((31, 30, 29), torch.float32, 2),
            ((32, 32, 32), torch.float32, 2), ((33, 32, 32), torch.float32, 0)]


@pytest.mark.parametrize("nsw", [1, 4, 5])
@pytest.mark.parametrize("st", [C.CS_FD, C.CS_Q1])
def test_resident_patches_equal_tiles_and_oracle(nsw, st):
    """Patches that fit in LDS run every sweep of a call in one launch; with
    the resident policy off the same patches take the tile kernels.  Both give
    the same iterate bit for bit, across the tier boundaries (16^3 small tier,
    24^3 FP64 and 32^3 FP32 large tier, one more point along x leaves it),
    non-cubic shapes, both parities and an odd layout, and equal the oracle."""
    res = {}
    for policy in (1, 0, 3):
        for dt in (torch.float64, torch.float32):
            C.cs_batch_resident_policy(st, C._DT[dt], policy)
        try:
            ps = [_patch(n, st, dt, i % 2, seed=2100 + 5 * i + st, layout="odd" if i % 5 == 4 else "aligned")
                  for i, (n, dt, _) in enumerate(RESIDENT)]
            bt = _batch(ps)
            per = [bt.sweeps_per_pass(i) for i in range(len(ps))]
            bt.gs(nsw)
            torch.cuda.synchronize()
            res[policy] = ([G.download(p["ug"]) for p in ps], per, ps)
            bt.close()
        finally:
            for dt in (torch.float64, torch.float32):
                C.cs_batch_resident_policy(st, C._DT[dt], 3)
    for i, (n, dt, tier) in enumerate(RESIDENT):
        assert (res[1][1][i] == 0) == (tier > 0), (n, dt)
        assert res[0][1][i] in (1, 2)  # tiles or, for small groups, colour passes
        assert (res[3][1][i] == 0) == (tier > 0)
        assert np.array_equal(res[1][0][i], res[0][0][i]), (n, dt)
        assert np.array_equal(res[3][0][i], res[0][0][i]), (n, dt)
        p = res[1][2][i]
        assert G.relmax(res[1][0][i], _oracle(p, nsw)) <= TOL[dt], (n, dt)
    with pytest.raises(C.ColstenError):
        C.cs_batch_resident_policy(st, 0, 8)


def test_resident_patch_alone_equals_patch_in_mix():
    """A resident patch gives the same bits alone and in a mix with tiled and
    other resident patches of both stencils."""
    probe_n, probe_seed = (20, 18, 22), 2300
    mix = [_patch(n, st, torch.float64, 0, seed=2310 + 3 * i + st)
           for i, n in enumerate([(8, 8, 8), (48, 48, 48), (24, 24, 24), (64, 20, 30)])
           for st in (C.CS_FD, C.CS_Q1)]
    for st in (C.CS_FD, C.CS_Q1):
        probe = _patch(probe_n, st, torch.float64, 1, seed=probe_seed + st)
        alone = _patch(probe_n, st, torch.float64, 1, seed=probe_seed + st)
        bm = _batch(mix[:3] + [probe] + mix[3:])
        bm.gs(7)
        ba = _batch([alone])
        assert ba.sweeps_per_pass(0) == 0
        ba.gs(7)
        torch.cuda.synchronize()
        assert torch.equal(probe["ug"], alone["ug"])
        bm.close()
        ba.close()


def _expected_per_pass(n, st, dt, mask):
    """Sweeps per pass the batch should report, from the documented tier rules
    (default tile and pass policies), for a batch too small to stream under
    bit 1 alone."""
    nx, ny, nz = n
    f64 = dt == torch.float64
    fd = st == C.CS_FD
    if mask & 1:
        elems = (nx + 2) * (ny + 2) * (nz + 2)
        per = (nx + 1) // 2 * ny * nz if fd else nx * ((ny + 1) // 2) * ((nz + 1) // 2)
        if elems <= 6144 and per <= 512 * (4 if fd else 2):
            return 0
        cap = 17600 if f64 else 40000
        pmax = (7 if fd else 4) if f64 else (16 if fd else 8)
        if elems <= cap and per <= 1024 * pmax:
            return 0
    if mask & 4 and nx * ny * nz <= 1 << 17:
        npl = 1 if fd else 2
        s_ = ((20000 if f64 else 40000) // ((nx + 2) * (ny + 2)) - 1 - npl) // 2
        pairs = (nx * ny + 1) // 2 if fd else nx * ((ny + 1) // 2)
        if s_ >= 2 and pairs <= 2048:
            return min(s_, 3 if fd else 2)
    return 2 if fd else 1


PLANES = [(32, 32, 32), (48, 48, 48), (25, 24, 24), (33, 9, 100), (40, 50, 3), (30, 30, 8),
          (55, 40, 30), (64, 64, 20), (80, 70, 9), (45, 44, 2)]


@pytest.mark.parametrize("nsw", [1, 4, 5, 7])
@pytest.mark.parametrize("st", [C.CS_FD, C.CS_Q1])
def test_plane_streamed_patches_equal_tiles_and_oracle(nsw, st, tiles_only_for_small_groups):
    """Patches whose cross-section fits several planes of LDS run every sweep
    of a call in one launch, streamed through z two or three sweeps per pass,
    in place; with that schedule off they take the tile kernels.  The reported
    sweeps per pass follow the tier rules, and both schedules give the same
    iterate bit for bit, equal to the oracle: cubic and flat shapes, a thin
    slab, both parities, an odd layout, FP64 and FP32."""
    cases = [(n, dt) for n in PLANES for dt in (torch.float64, torch.float32)]
    res = {}
    for policy in (7, 1):
        for dt in (torch.float64, torch.float32):
            C.cs_batch_resident_policy(st, C._DT[dt], policy)
        try:
            ps = [_patch(n, st, dt, i % 2, seed=2400 + 7 * i + st, layout="odd" if i % 4 == 3 else "aligned")
                  for i, (n, dt) in enumerate(cases)]
            bt = _batch(ps)
            per = [bt.sweeps_per_pass(i) for i in range(len(ps))]
            bt.gs(nsw)
            torch.cuda.synchronize()
            res[policy] = ([G.download(p["ug"]) for p in ps], per, ps)
            bt.close()
        finally:
            for dt in (torch.float64, torch.float32):
                C.cs_batch_resident_policy(st, C._DT[dt], 3)
    streamed = 0
    for i, (n, dt) in enumerate(cases):
        for policy in (7, 1):
            assert res[policy][1][i] == _expected_per_pass(n, st, dt, policy), (n, dt, policy)
        streamed += _expected_per_pass(n, st, dt, 7) != _expected_per_pass(n, st, dt, 1)
        assert np.array_equal(res[7][0][i], res[1][0][i]), (n, dt)
        assert G.relmax(res[7][0][i], _oracle(res[7][2][i], nsw)) <= TOL[dt], (n, dt)
    assert streamed >= 8


def test_streaming_needs_a_patch_per_compute_unit(tiles_only_for_small_groups):
    """Under the default mask the streamable patches of a stencil and dtype
    are streamed only when the batch holds one per compute unit: a batch of
    that many streams every one of them, a batch of one fewer sweeps them all
    with the tile kernels, and the shared patches end bit for bit equal, and
    equal to the oracle."""
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    n = (26, 26, 30)  # beyond the resident tiers, streamable
    ps = [_patch(n, C.CS_FD, torch.float64, i % 2, seed=2600 + i) for i in range(ncu)]
    bt_all = _batch(ps)
    assert {bt_all.sweeps_per_pass(i) for i in range(ncu)} == {3}
    bt_all.gs(5)
    torch.cuda.synchronize()
    got_all = [G.download(ps[i]["ug"]) for i in (0, 1, ncu - 2)]
    bt_all.close()
    qs = [_patch(n, C.CS_FD, torch.float64, i % 2, seed=2600 + i) for i in range(ncu - 1)]
    bt_less = _batch(qs)
    assert {bt_less.sweeps_per_pass(i) for i in range(ncu - 1)} == {2}
    bt_less.gs(5)
    torch.cuda.synchronize()
    for k, i in enumerate((0, 1, ncu - 2)):
        assert np.array_equal(got_all[k], G.download(qs[i]["ug"])), i
    bt_less.close()
    assert G.relmax(got_all[1], _oracle(_patch(n, C.CS_FD, torch.float64, 1, seed=2601), 5)) <= 1e-13


@pytest.mark.parametrize("nsw", [1, 4, 5])
def test_colour_passes_equal_tiles_bitwise(nsw):
    """The same patches swept by the colour passes (every group) and by the
    tile kernels (none) end bit for bit equal: both stencils, FP64 and FP32,
    both parities, ragged and odd layouts, single and paired tile classes."""
    shapes = [(1, 1, 1), (5, 7, 3), (17, 9, 12), (33, 20, 18), (70, 13, 65), (64, 64, 40),
              (40, 66, 9), (123, 31, 17)]
    res = {}
    for colour in (1 << 40, 0):
        _set_policies(resident=0, colour=colour)
        try:
            ps = [_patch(n, st, dt, (i + st) % 2, seed=2700 + 3 * i + st, layout="odd" if i % 3 == 2 else "aligned")
                  for i, n in enumerate(shapes) for st in (C.CS_FD, C.CS_Q1)
                  for dt in (torch.float64, torch.float32)]
            bt = _batch(ps)
            per = {bt.sweeps_per_pass(i) for i in range(len(ps))}
            assert per == ({1} if colour else {1, 2})
            bt.gs(nsw)
            torch.cuda.synchronize()
            res[colour] = [G.download(p["ug"]) for p in ps]
            bt.close()
        finally:
            _set_policies()
    for a, b in zip(res[1 << 40], res[0]):
        assert np.array_equal(a, b)
