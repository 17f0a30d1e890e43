"""Autotuner for the batched-patch tile shapes and colour schedules, and for
the automatic schedule of single grids.

The tile policy and the colour schedule are timed on a mix of patches of
arbitrary shape (axis lengths log-uniform in [16, 128], aspect at most 4, as a
request stream draws them), since the small cubic patches are swept resident
or streamed and the tiles serve the rest: each candidate pair of thresholds
(small_max, mid_max) of cs_batch_tile_policy is timed on the mix and the
fastest is set; for the 7-point stencil the large tiles' two sweeps per pass
are then timed against one sweep per pass on the same mix and the faster is
set with cs_batch_pass_policy.  Groups of the 1, 2, 4, 8 and 16 largest
patches of the mix are timed with the tiles and with the colour passes, and
the colour-pass threshold of cs_batch_colour_policy is set past the largest
group on which the colour passes won.  Last, the resident schedules are timed on a
mix of cubic patches of every edge class (8 to 64) with the resident masks 3
(whole patches in LDS, plane streaming for large classes), 1 (whole patches
only) and 0 (tiles only), and the fastest mask is set with
cs_batch_resident_policy.  Every schedule gives the same iterate.  Results are
cached as JSON keyed by GPU architecture, stencil and dtype
(COLSTEN_TUNE_CACHE, default ~/.cache/colsten_tune.json), so later processes
apply them without re-timing.

Single grids (tune_grid): cubic grids from 8^3 to 256^3 are swept under each
schedule of the automatic mode -- every sweep in one workgroup, one launch per
colour, fused passes of one or of two sweeps -- and the size limits of
cs_grid_schedule_policy are set where the fastest schedule changes.
"""
import json
import os
import sys

import torch

from . import colsten as C
from . import inputs as I

VARIANT_TILES = {C.CS_FD: ["16x16", "32x16", "64x16"], C.CS_Q1: ["16x8", "32x16", "64x16"]}
# candidate (small_max, mid_max): large tiles only, middle tiles up to 40 or
# 64 points along x, and small tiles up to 16 as well
TILE_CANDIDATES = [(0, 0), (0, 40), (0, 64), (16, 40)]


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


def shape_mix(points_target, seed=13):
    """Patch shapes of a request stream (log-uniform axes in [16, 128], aspect
    at most 4) up to about points_target interior points."""
    shapes, total = [], 0
    for r in I.request_stream(seed, 4096, 1000.0):
        shapes.append(tuple(r.n))
        total += r.n[0] * r.n[1] * r.n[2]
        if total >= points_target:
            break
    return shapes


def cube_mix(edges, points_target):
    """Cubic patches cycling through edges (equal counts) up to about
    points_target interior points."""
    shapes, total = [], 0
    while not shapes or total < points_target:
        e = edges[len(shapes) % len(edges)]
        shapes.append((e, e, e))
        total += e ** 3
    return shapes


def _time_shapes(shapes, stencil, dtype, sweeps):
    """GLUP/s of one batch of the given shapes under the current policies."""
    ps = []
    for n in shapes:
        u = C.empty_grid(n, dtype=dtype)
        b = C.empty_grid(n, dtype=dtype)
        b.fill_(1.0)
        ps.append((u, b, C.grid_like(u), stencil, 1.0 / (max(n) + 1), 0))
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
    total = sum(n[0] * n[1] * n[2] for n in shapes)
    return total * sweeps / (ms * 1e-3) / 1e9


def _log(msg):
    print("tune: " + msg, file=sys.stderr, flush=True)


def _restore_batch_defaults(stencil, dt):
    C.cs_batch_tile_policy(stencil, dt, 0, 0)
    C.cs_batch_pass_policy(stencil, dt, 1)
    C.cs_batch_colour_policy(stencil, dt, -1)
    C.cs_batch_resident_policy(stencil, dt, 3)


def tune(stencil, dtype=torch.float64, edges=(8, 16, 24, 32, 48, 64), points_target=1 << 24,
         sweeps=10, save=True):
    """Time the candidate policies; returns the record and applies the
    fastest (the defaults stay in force if a timing fails)."""
    try:
        return _tune(stencil, dtype, edges, points_target, sweeps, save)
    except BaseException:
        _restore_batch_defaults(stencil, C._DT[dtype])
        raise


def _tune(stencil, dtype, edges, points_target, sweeps, save):
    dt = C._DT[dtype]
    mix = shape_mix(points_target)
    C.cs_batch_resident_policy(stencil, dt, 3)
    C.cs_batch_pass_policy(stencil, dt, 1)
    C.cs_batch_colour_policy(stencil, dt, 0)  # the tiles themselves are timed first
    tiles = {}
    for cand in TILE_CANDIDATES:
        C.cs_batch_tile_policy(stencil, dt, *cand)
        tiles[cand] = _time_shapes(mix, stencil, dtype, sweeps)
        _log("shape mix, tile thresholds %s: %.1f GLUP/s" % (cand, tiles[cand]))
    small_max, mid_max = max(tiles, key=lambda c: tiles[c])
    C.cs_batch_tile_policy(stencil, dt, small_max, mid_max)
    passes = {True: tiles[(small_max, mid_max)]}
    if stencil == C.CS_FD:
        C.cs_batch_pass_policy(stencil, dt, 0)
        passes[False] = _time_shapes(mix, stencil, dtype, sweeps)
        _log("shape mix, one sweep per pass: %.1f GLUP/s" % passes[False])
    pair = passes[True] >= passes.get(False, 0.0)
    C.cs_batch_pass_policy(stencil, dt, pair)
    # colour passes for small groups: groups of the k largest patches of the
    # mix, tiles against colour passes; the threshold lies past the largest
    # group on which the colour passes won
    big = sorted(mix, key=lambda n: -n[0] * n[1] * n[2])
    small, colour_max = {}, 0
    for k in (1, 2, 4, 8, 16):
        grp = big[:k]
        pts = sum(n[0] * n[1] * n[2] for n in grp)
        r = []
        for cm in (0, 1 << 40):
            C.cs_batch_colour_policy(stencil, dt, cm)
            r.append(_time_shapes(grp, stencil, dtype, sweeps))
        small[k] = (pts, r)
        _log("%d largest patches (%d points): tiles %.1f, colour passes %.1f GLUP/s" % (k, pts, r[0], r[1]))
    for k in (1, 2, 4, 8, 16):
        pts, (tile_r, col_r) = small[k]
        if col_r <= tile_r:
            break
        nxt = small.get(2 * k)
        colour_max = (pts + nxt[0]) // 2 if nxt else pts + 1
    C.cs_batch_colour_policy(stencil, dt, colour_max)
    cubes = cube_mix(list(edges), 8 * points_target)
    res = {}
    for r in (3, 1, 0):
        C.cs_batch_resident_policy(stencil, dt, r)
        res[r] = _time_shapes(cubes, stencil, dtype, sweeps)
        _log("cube mix of edges %s, resident mask %d: %.1f GLUP/s" % (list(edges), r, res[r]))
    resident = max(res, key=lambda r: res[r])
    C.cs_batch_resident_policy(stencil, dt, resident)
    rec = {"small_max": small_max, "mid_max": mid_max, "pair_large": bool(pair),
           "colour_max_points": colour_max, "resident": resident,
           "glups_small_groups": {str(k): {"points": v[0], "tiles": round(v[1][0], 2),
                                           "colour_passes": round(v[1][1], 2)} for k, v in small.items()},
           "glups_shape_mix_tiles": {"%d,%d" % c: round(v, 2) for c, v in tiles.items()},
           "glups_shape_mix_passes": {("two_sweeps" if p else "one_sweep") + "_per_pass": round(v, 2)
                                      for p, v in passes.items()},
           "glups_cube_mix_resident": {"mask_%d" % r: round(v, 2) for r, v in res.items()},
           "shape_mix_patches": len(mix), "tiles": VARIANT_TILES[stencil]}
    if save:
        _save(_key(stencil, dtype), rec)
    return rec


# ---- single grids ------------------------------------------------------------

GRID_EDGES = (8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256)
NEVER = 1 << 62


def _grid_key(stencil, dtype):
    return "grid/" + _key(stencil, dtype)


def _time_grid(n, stencil, dtype, sweeps, schedule, reps=3):
    """Seconds for `sweeps` sweeps of a cubic n^3 grid under one schedule of
    the automatic mode: 'block' (one workgroup), 'colour' (one launch per
    colour), 'one' / 'two' (fused passes, one or two sweeps per pass)."""
    dt = C._DT[dtype]
    big = NEVER
    pol = {"block": (big, 0, big), "colour": (0, big, big), "one": (0, 0, big), "two": (0, 0, 0)}[schedule]
    C.cs_grid_schedule_policy(stencil, dt, *pol)
    u = C.empty_grid((n, n, n), dtype=dtype)
    b = C.empty_grid((n, n, n), dtype=dtype)
    b.fill_(1.0)
    tmp = C.grid_like(u)
    g = C.Grid(u, b, dim=3, stencil=stencil, h=1.0 / (n + 1))
    try:
        if schedule == "two" and g.sweeps_per_pass() != 2:
            return None
        g.gs(2, tmp=tmp)
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            g.gs(sweeps, tmp=tmp)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) * 1e-3
            best = t if best is None else min(best, t)
        return best
    finally:
        g.close()


def tune_grid(stencil, dtype=torch.float64, edges=GRID_EDGES, sweeps=20, block_edge_max=48, save=True):
    """Time the automatic mode's schedules of cs_gs_sweeps on cubic grids of
    the given edges, derive the size limits of cs_grid_schedule_policy from
    the fastest schedule per edge, apply them and cache them."""
    dt = C._DT[dtype]
    table = {}
    try:
        for n in edges:
            row = {}
            for sch in ("block", "colour", "one", "two"):
                if sch == "block" and n > block_edge_max:
                    continue
                t = _time_grid(n, stencil, dtype, sweeps, sch)
                if t is not None:
                    row[sch] = n ** 3 * sweeps / t / 1e9
            table[n] = row
            _log("grid %d^3: %s GLUP/s" % (n, {k: round(v, 1) for k, v in row.items()}))
    finally:
        C.cs_grid_schedule_policy(stencil, dt, -1, -1, -1)

    def cut(lo_edge, hi_edge):
        # a limit between two measured sizes (geometric mean of the point counts)
        return int((lo_edge ** 3 * hi_edge ** 3) ** 0.5)

    def limit_below(wins):
        # the largest edge that wins, and every smaller one too; the limit lies
        # between it and the next edge
        last = None
        for i, n in enumerate(edges):
            if not wins(n):
                break
            last = i
        if last is None:
            return 0
        return cut(edges[last], edges[last + 1]) if last + 1 < len(edges) else NEVER

    fused = lambda n: max(v for k, v in table[n].items() if k in ("one", "two"))  # noqa: E731
    block_max = limit_below(lambda n: "block" in table[n] and
                            table[n]["block"] >= max(v for k, v in table[n].items()))
    colour_max = limit_below(lambda n: table[n]["colour"] >= fused(n))
    two_min = NEVER
    for i in range(len(edges) - 1, -1, -1):
        n = edges[i]
        if table[n].get("two", 0.0) > table[n]["one"]:
            two_min = cut(edges[i - 1], n) if i > 0 else 0
        else:
            break
    C.cs_grid_schedule_policy(stencil, dt, block_max, colour_max, two_min)
    rec = {"block_max": block_max, "colour_max": colour_max, "two_min": two_min,
           "glups": {str(n): {k: round(v, 2) for k, v in row.items()} for n, row in table.items()},
           "sweeps": sweeps}
    if save:
        _save(_grid_key(stencil, dtype), rec)
    return rec


def apply_cached_grid(stencil, dtype=torch.float64):
    """Apply a cached single-grid schedule policy if there is one; returns it
    (or None)."""
    rec = _load(_grid_key(stencil, dtype))
    if rec:
        C.cs_grid_schedule_policy(stencil, C._DT[dtype], rec["block_max"], rec["colour_max"], rec["two_min"])
    return rec


def _save(key, rec):
    path = cache_path()
    data = {}
    if os.path.exists(path):
        try:
            data = json.load(open(path))
        except ValueError:
            data = {}
    data[key] = rec
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1)
    os.replace(tmp, path)


def _load(key):
    path = cache_path()
    if not os.path.exists(path):
        return None
    try:
        return json.load(open(path)).get(key)
    except ValueError:
        return None


def apply_cached(stencil, dtype=torch.float64):
    """Apply a cached batch policy if there is one; returns it (or None)."""
    rec = _load(_key(stencil, dtype))
    if rec:
        C.cs_batch_tile_policy(stencil, C._DT[dtype], rec["small_max"], rec["mid_max"])
        C.cs_batch_pass_policy(stencil, C._DT[dtype], rec.get("pair_large", True))
        C.cs_batch_colour_policy(stencil, C._DT[dtype], rec.get("colour_max_points", -1))
        res = rec.get("resident", 3)
        C.cs_batch_resident_policy(stencil, C._DT[dtype], 3 if res is True else int(res))
    return rec
