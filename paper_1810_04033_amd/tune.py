"""Autotuner for the batched-patch tile shapes and colour schedule.

For each patch edge class it times the batched Gauss-Seidel sweep with each
tile variant (small, middle, large tiles) on a batch of equal patches large
enough to fill the GPU, picks the fastest variant per edge, and turns the
picks into the size thresholds of cs_batch_tile_policy.  For the 7-point
stencil the large tiles are timed with two sweeps per pass and with one, per
edge and on a batch mixing (in equal counts) the edges that pick them, and the
schedule that is faster on the mix is set with cs_batch_pass_policy (both give
the same iterate; batches of equal patches are chunked differently from mixed
ones, so the mix decides).  Last, the patches small enough to be swept
resident in one workgroup's LDS (all sweeps in one launch) are timed that way
and with the chosen tiles, on a mix of those edges, and the faster schedule is
set with cs_batch_resident_policy.  Results are cached
as JSON keyed by GPU architecture, stencil and dtype (COLSTEN_TUNE_CACHE,
default ~/.cache/colsten_tune.json), so later processes apply them without
re-timing.
"""
import json
import os
import sys

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


def _time_batch(edge, stencil, dtype, variant, points_target, sweeps, pair=True):
    # force one variant (and schedule) for every edge
    C.cs_batch_tile_policy(stencil, C._DT[dtype], 1 << 30 if variant == 0 else 0,
                           1 << 30 if variant <= 1 else 0)
    return _time_edges([edge], stencil, dtype, points_target, sweeps, pair)


def _time_edges(edges, stencil, dtype, points_target, sweeps, pair, resident=False):
    """GLUP/s of a batch of cubic patches cycling through edges (equal counts)
    up to about points_target points, under the current tile policy."""
    C.cs_batch_pass_policy(stencil, C._DT[dtype], pair)
    C.cs_batch_resident_policy(stencil, C._DT[dtype], int(resident))
    sizes, total = [], 0
    while not sizes or total < points_target:
        sizes.append(edges[len(sizes) % len(edges)])
        total += sizes[-1] ** 3
    ps = []
    for edge in sizes:
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
    return total * sweeps / (ms * 1e-3) / 1e9


def tune(stencil, dtype=torch.float64, edges=(8, 16, 24, 32, 48, 64), points_target=1 << 24,
         sweeps=10, save=True):
    """Time every variant on every edge class; returns the record and applies
    the resulting policy."""
    table, single = {}, {}
    for e in edges:
        table[e] = [_time_batch(e, stencil, dtype, v, points_target, sweeps) for v in range(3)]
        # the large tiles with one sweep per pass, where they can compete
        if stencil == C.CS_FD and table[e][2] >= 0.75 * max(table[e][:2]):
            single[e] = _time_batch(e, stencil, dtype, 2, points_target, sweeps, pair=False)
        print("tune: edge %d: %s%s" % (e, [round(x, 1) for x in table[e]],
                                       " one sweep per pass %.1f" % single[e] if e in single else ""),
              file=sys.stderr, flush=True)
    # the large tiles count with their faster schedule
    rate = {e: table[e][:2] + [max(table[e][2], single.get(e, 0.0))] for e in edges}
    best = {e: max(range(3), key=lambda v: rate[e][v]) for e in edges}
    # thresholds: the largest edge whose best variant is 0, then <= 1
    small_max = max([e for e in edges if best[e] == 0], default=0)
    mid_max = max([e for e in edges if best[e] <= 1] + [small_max])
    large = [e for e in edges if best[e] == 2]
    C.cs_batch_tile_policy(stencil, C._DT[dtype], small_max, mid_max)
    # schedule of the large tiles, timed on a mix of the edges that use them,
    # sized like a large batch (the z-chunking of a batch depends on its size)
    mix = {}
    if stencil == C.CS_FD and large:
        for p in (True, False):
            mix[p] = _time_edges(large, stencil, dtype, 8 * points_target, sweeps, p)
            print("tune: mix of edges %s, %s per pass: %.1f GLUP/s"
                  % (large, "two sweeps" if p else "one sweep", mix[p]), file=sys.stderr, flush=True)
    pair = not mix or mix[True] >= mix[False]
    C.cs_batch_pass_policy(stencil, C._DT[dtype], pair)
    # the resident schedule, on a mix of the edges it takes
    fits = [e for e in edges if _resident_fits(e, stencil, dtype)]
    res = {}
    if fits:
        for r in (True, False):
            res[r] = _time_edges(fits, stencil, dtype, points_target, sweeps, pair, resident=r)
            print("tune: mix of edges %s, %s: %.1f GLUP/s" % (fits, "resident" if r else "tiles", res[r]),
                  file=sys.stderr, flush=True)
    resident = bool(res) and res[True] >= res[False]
    C.cs_batch_resident_policy(stencil, C._DT[dtype], int(resident))
    rec = {"small_max": small_max, "mid_max": mid_max, "pair_large": bool(pair),
           "resident": resident,
           "glups_resident_mix": {("resident" if r else "tiles"): round(v, 2) for r, v in res.items()},
           "glups": {str(e): [round(x, 2) for x in table[e]] for e in edges},
           "glups_large_one_sweep_per_pass": {str(e): round(single[e], 2) for e in single},
           "glups_large_mix": {("two_sweeps" if p else "one_sweep") + "_per_pass": round(v, 2)
                               for p, v in mix.items()},
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
        C.cs_batch_pass_policy(stencil, C._DT[dtype], rec.get("pair_large", True))
        C.cs_batch_resident_policy(stencil, C._DT[dtype], int(rec.get("resident", True)))
    return rec


def _resident_fits(edge, stencil, dtype):
    """Whether a cubic patch of this edge is swept resident in LDS (asked of
    the library through a one-patch batch)."""
    C.cs_batch_resident_policy(stencil, C._DT[dtype], 1)
    u = C.empty_grid((edge,) * 3, dtype=dtype)
    bt = C.Batch([(u, C.grid_like(u), C.grid_like(u), stencil, 1.0 / (edge + 1), 0)])
    fits = bt.sweeps_per_pass(0) == 0
    bt.close()
    return fits
