"""The batch autotuner on the GPU: it times its candidates, applies and
caches a valid policy, and a later apply_cached restores it."""
import json

import pytest
import torch

from paper_1810_04033_amd import colsten as C
from paper_1810_04033_amd import tune as T

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
