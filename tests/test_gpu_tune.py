"""The autotuners on the GPU: the batch tuner and the single-grid tuner time
their candidates, apply and cache a valid policy, and a later apply restores
it; every schedule the single-grid policy selects gives the oracle's iterate."""
import json

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1810_04033_amd import colsten as C
from paper_1810_04033_amd import tune as T

import gpu_util as G

pytestmark = pytest.mark.gpu


def test_tune_applies_and_caches_a_policy(tmp_path, monkeypatch):
    monkeypatch.setenv("COLSTEN_TUNE_CACHE", str(tmp_path / "tune.json"))
    try:
        for st in (C.CS_FD, C.CS_Q1):
            rec = T.tune(st, torch.float64, points_target=1 << 21, sweeps=2)
            assert (rec["small_max"], rec["mid_max"]) in T.TILE_CANDIDATES
            assert rec["resident"] in (0, 1, 3)
            assert set(rec["glups_shape_mix_tiles"]) == {"%d,%d" % c for c in T.TILE_CANDIDATES}
            assert all(v > 0 for v in rec["glups_shape_mix_tiles"].values())
            assert (len(rec["glups_shape_mix_passes"]) == 2) == (st == C.CS_FD)
            assert rec["colour_max_points"] >= 0 and len(rec["glups_small_groups"]) == 5
            data = json.load(open(tmp_path / "tune.json"))
            assert data[T._key(st, torch.float64)] == json.loads(json.dumps(rec))
            assert T.apply_cached(st, torch.float64) == data[T._key(st, torch.float64)]
        assert T.apply_cached(C.CS_FD, torch.float32) is None
    finally:
        for st in (C.CS_FD, C.CS_Q1):
            for dt in (C.CS_F64, C.CS_F32):
                C.cs_batch_tile_policy(st, dt, 0, 0)
                C.cs_batch_pass_policy(st, dt, 1)
                C.cs_batch_resident_policy(st, dt, 3)
                C.cs_batch_colour_policy(st, dt, -1)


NP = {torch.float64: np.float64, torch.float32: np.float32}
BIG = 1 << 62
SCHEDULES = {"block": (BIG, 0, BIG), "colour": (0, BIG, BIG), "one": (0, 0, BIG), "two": (0, 0, 0)}


@pytest.mark.parametrize("n", [(12, 12, 12), (40, 33, 37)], ids=lambda p: "x".join(map(str, p)))
@pytest.mark.parametrize("stencil", [C.CS_FD, C.CS_Q1], ids=["fd", "q1"])
@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_grid_schedule_policy_same_iterate(n, stencil, dt):
    """Every schedule the single-grid policy can select (one workgroup, one
    launch per colour, fused passes of one or two sweeps) gives the oracle's
    iterate bit for bit, odd layout, parity 1, 6 sweeps."""
    u, b = G.case(3, n, seed=3700 + stencil + sum(n))
    h = 1.0 / (max(n) + 1)
    uo, bo = u.astype(NP[dt]), b.astype(NP[dt])
    O.gs_sweeps(uo, bo, 6, dim=3, stencil=stencil, h=h, parity=1)
    try:
        for name, pol in SCHEDULES.items():
            C.cs_grid_schedule_policy(stencil, C._DT[dt], *pol)
            ug, bg = G.upload(u, dt, layout="odd"), G.upload(b, dt, layout="odd")
            g = C.Grid(ug, bg, dim=3, stencil=stencil, h=h, parity=1)
            if name == "two":
                assert g.sweeps_per_pass() == 2
            elif name == "one":
                assert g.sweeps_per_pass() == 1
            g.gs(6, tmp=C.grid_like(ug))
            torch.cuda.synchronize()
            assert np.array_equal(ug.detach().cpu().numpy(), uo), name
            g.close()
    finally:
        C.cs_grid_schedule_policy(stencil, C._DT[dt], -1, -1, -1)
    with pytest.raises(C.ColstenError):
        C.cs_grid_schedule_policy(2, 0, -1, -1, -1)


def test_tune_grid_applies_and_caches(tmp_path, monkeypatch):
    monkeypatch.setenv("COLSTEN_TUNE_CACHE", str(tmp_path / "tune.json"))
    try:
        rec = T.tune_grid(C.CS_FD, torch.float64, edges=(8, 16, 32, 64), sweeps=4, block_edge_max=16)
        assert set(rec["glups"]) == {"8", "16", "32", "64"}
        assert all(v > 0 for row in rec["glups"].values() for v in row.values())
        assert "block" in rec["glups"]["8"] and "block" not in rec["glups"]["32"]
        assert 0 <= rec["block_max"] and 0 <= rec["colour_max"] and 0 <= rec["two_min"]
        assert T.apply_cached_grid(C.CS_FD, torch.float64) == json.loads(json.dumps(rec))
        assert T.apply_cached_grid(C.CS_Q1, torch.float64) is None
    finally:
        C.cs_grid_schedule_policy(C.CS_FD, C.CS_F64, -1, -1, -1)
