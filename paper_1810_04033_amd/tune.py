"""Autotuner for the batched-patch tile shapes.

For each patch edge class it times the batched Gauss-Seidel sweep with each
tile variant (small, middle, large tiles) on a batch of equal patches large
enough to fill the GPU, picks the fastest variant per edge, and turns the
picks into the size thresholds of cs_batch_tile_policy.  Results are cached
as JSON keyed by GPU architecture, stencil and dtype (COLSTEN_TUNE_CACHE,
default ~/.cache/colsten_tune.json), so later processes apply them without
re-timing.
"""
import json
import os

import torch

from . import colsten as C

VARIANT_TILES = {C.CS_FD: ["16x16", "32x16", "64x16"], C.CS_Q1: ["16x8", "32x16", "64x16"]}


def cache_path():
    return os.environ.get("COLSTEN_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "colsten_tune.json"))


def _arch():
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _key(stencil, dtype):
    return "%s/%s/%s" % (_arch(), "fd" if stencil == C.CS_FD else "q1",
                         "f64" if dtype == torch.float64 else "f32")


def _time_batch(edge, stencil, dtype, variant, points_target, sweeps):
    # force one variant for every edge
    C.cs_batch_tile_policy(stencil, C._DT[dtype], 1 << 30 if variant == 0 else 0,
                           1 << 30 if variant <= 1 else 0)
    count = max(1, points_target // edge ** 3)
    ps = []
    for _ in range(count):
        u = C.empty_grid((edge,) * 3, dtype=dtype)
        b = C.empty_grid((edge,) * 3, dtype=dtype)
        b.fill_(1.0)
        ps.append((u, b, C.grid_like(u), stencil, 1.0 / (edge + 1), 0))
    bt = C.Batch(ps)
    bt.gs(2)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    bt.gs(sweeps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    bt.close()
    return count * edge ** 3 * sweeps / (ms * 1e-3) / 1e9


def tune(stencil, dtype=torch.float64, edges=(8, 16, 24, 32, 48, 64), points_target=1 << 24,
         sweeps=10, save=True):
    """Time every variant on every edge class; returns the record and applies
    the resulting policy."""
    table = {}
    for e in edges:
        table[e] = [_time_batch(e, stencil, dtype, v, points_target, sweeps) for v in range(3)]
    best = {e: max(range(3), key=lambda v: table[e][v]) for e in edges}
    # thresholds: the largest edge whose best variant is 0, then <= 1
    small_max = max([e for e in edges if best[e] == 0], default=0)
    mid_max = max([e for e in edges if best[e] <= 1] + [small_max])
    C.cs_batch_tile_policy(stencil, C._DT[dtype], small_max, mid_max)
    rec = {"small_max": small_max, "mid_max": mid_max,
           "glups": {str(e): [round(x, 2) for x in table[e]] for e in edges},
           "tiles": VARIANT_TILES[stencil]}
    if save:
        path = cache_path()
        data = {}
        if os.path.exists(path):
            try:
                data = json.load(open(path))
            except ValueError:
                data = {}
        data[_key(stencil, dtype)] = rec
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1)
        os.replace(tmp, path)
    return rec


def apply_cached(stencil, dtype=torch.float64):
    """Apply a cached policy if there is one; returns it (or None)."""
    path = cache_path()
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(_key(stencil, dtype))
    except ValueError:
        return None
    if rec:
        C.cs_batch_tile_policy(stencil, C._DT[dtype], rec["small_max"], rec["mid_max"])
    return rec
