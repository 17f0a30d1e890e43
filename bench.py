"""Benchmark of the coloured stencil sweeps on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload (one step): the 3D Poisson problem on a 256^3 interior grid, h = 1/257,
FP64, zero Dirichlet boundary, seeded uniform[-1,1) right-hand side, u0 = 0:
  100 red-black Gauss-Seidel sweeps with the 7-point stencil,
  100 8-colour Gauss-Seidel sweeps with the 27-point trilinear stencil,
  100 weighted Jacobi sweeps (omega = 2/3) with each stencil,
  then the residual norms of both Gauss-Seidel results.
value = grid-point updates per second over the 400 sweeps (the residual time is
inside the step).  Inputs are resident in HBM before timing starts.

Printed: one JSON line with the throughput, a per-row breakdown, the roofline
of the dominant kernel (algorithmic bytes per launch over its mean launch
duration, timed with HIP events on the launch stream inside the timed region)
and the oracle timed on the host for a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N = 256
H = 1.0 / 257
SWEEPS = 100
OMEGA = 2.0 / 3.0
BYTES_PER_UPDATE = 24  # FP64: read u, read b, write u (single sweep, no reuse)

ROWS = ("gs_fd7", "gs_q1_27", "jacobi_fd7", "jacobi_q1_27", "residuals")


def _args():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-growth", action="store_true",
                   help="poisson3d: leave out the batched-patch and serving figures of the line")
    p.add_argument("--per-colour", action="store_true",
                   help="run the GS rows as one launch per colour pass (no work array)")
    p.add_argument("--workload", default="poisson3d",
                   choices=["poisson3d", "patches", "refine", "serve", "expensive", "orderings",
                            "multigrid", "slab", "calib"],
                   help="poisson3d (default, the headline line); patches: 4096 batched patches; "
                        "refine: FP32 sweeps in FP64 refinement to 1e-10; serve: request stream; "
                        "expensive: sweeps with the S(k) stencil cost; orderings: lexicographic "
                        "wavefront GS beside coloured GS; multigrid: V-cycles with the coloured "
                        "smoother to 1e-10; slab: the sweep rows on one GPU's z-slab; calib: a "
                        "plain 1 GiB device copy for scaling rocprofv3's byte counters")
    p.add_argument("--tune", action="store_true", help="patches: run the tile autotuner first")
    p.add_argument("--patch-baselines", default="per_colour,fused_per_patch",
                   help="patches: the per-patch launch schedules timed beside the batch "
                        "(comma list of per_colour, fused_per_patch; empty for none)")
    p.add_argument("--serve-count", type=int, default=300, help="serve: requests in the stream")
    p.add_argument("--refine-n", type=int, default=512, help="refine: interior edge")
    p.add_argument("--mg-n", type=int, default=255, help="multigrid: interior edge, 2^m - 1")
    p.add_argument("--mg-gs-compare", type=int, default=1,
                   help="multigrid: also solve with the coloured sweeps alone (1) or not (0)")
    p.add_argument("--slab", default="512,512,64;256,256,32",
                   help="slab: interior shapes nx,ny,nz separated by ';' (one GPU's eighth of "
                        "512^3 and of 256^3 by default)")
    p.add_argument("--slab-dtype", default="f64", choices=["f64", "f32"],
                   help="slab: element type of the sweeps")
    p.add_argument("--slab-rows", default="gs_fd7,jacobi_fd7,gs_q1_27,jacobi_q1_27",
                   help="slab: the sweep rows to run")
    p.add_argument("--slab-sweeps", type=int, default=100, help="slab: sweeps per row")
    return p.parse_args()


def _source_sha(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic(kernel_key, sha):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except ValueError:
        return None
    rec = data.get(kernel_key)
    if not rec or rec.get("source_sha") != sha:
        return None
    return rec.get("hbm_bytes_per_launch")


def _omp_threads():
    """Threads of the OpenMP oracle: OMP_NUM_THREADS if set, else the cores
    this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


CPU_SWEEPS = 2  # sweeps of each kind in the host sample


def _host_cpu():
    """Model name of the host CPU and the cores this process may use."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": name, "cores_available": len(os.sched_getaffinity(0))}


def cpu_baseline(openmp=False):
    """The oracle on the host: two sweeps of each kind plus both residuals at
    the full 256^3 size (about 10 s), single thread; with openmp, the sweeps alone with
    the same oracle source built with OpenMP (one parallel loop per colour, the
    paper's BSP colouring of Sec. 3) on the host cores (the residual's
    fixed-order sums are sequential, so they are left out of that sample)."""
    import numpy as np
    from oracle import oracle as O
    from paper_1810_04033_amd import inputs as I

    O.set_openmp(openmp)
    b = I.halo_array(I.uniform_field(2, (N, N, N)))
    t0 = time.perf_counter()
    for st in (O.FD, O.Q1):
        u = I.halo_array(np.zeros((N, N, N)))
        O.gs_sweeps(u, b, CPU_SWEEPS, dim=3, stencil=st, h=H)
        if not openmp:
            O.residual(u, b, dim=3, stencil=st, h=H)
        uj = I.halo_array(np.zeros((N, N, N)))
        O.jacobi_sweeps(uj, b, CPU_SWEEPS, OMEGA, dim=3, stencil=st, h=H)
    dt = time.perf_counter() - t0
    O.set_openmp(False)
    if openmp:
        return {"value": 4 * CPU_SWEEPS * N ** 3 / dt / 1e9, "unit": "GLUP/s", "cores": _omp_threads(),
                "kind": "oracle, OpenMP build",
                "sample": "two sweeps of each of the four sweep kinds on the full 256^3 grid (no "
                          "residuals), the oracle built with -fopenmp (a parallel loop per colour "
                          "and per Jacobi sweep), %.1f s" % dt}
    return {"value": 4 * CPU_SWEEPS * N ** 3 / dt / 1e9, "unit": "GLUP/s", "cores": 1, "kind": "oracle",
            "host": _host_cpu(),
            "sample": "two sweeps of each of the four sweep kinds plus both residual norms on the "
                      "full 256^3 grid, sequential C oracle, %.1f s" % dt}


def run_poisson3d(a):
    import numpy as np
    import torch

    from paper_1810_04033_amd import colsten as C
    from paper_1810_04033_amd import inputs as I

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    n3 = (N, N, N)
    b_host = I.halo_array(I.uniform_field(2, n3))
    b = C.empty_grid(n3)
    b.copy_(torch.from_numpy(b_host))
    del b_host
    tmp = C.empty_grid(n3)
    grids = {}
    for name, st in (("fd7", C.CS_FD), ("q1_27", C.CS_Q1)):
        u_gs = C.empty_grid(n3)
        u_j = C.empty_grid(n3)
        grids[name] = (C.Grid(u_gs, b, dim=3, stencil=st, h=H), C.Grid(u_j, b, dim=3, stencil=st, h=H))
    norms = torch.zeros(2, 3, dtype=torch.float64, device="cuda")
    gs_tmp = None if a.per_colour else tmp
    fused_rows = {name: (gs_tmp is not None and grids[name][0].fused) for name in grids}

    def step(ev=None):
        for g_gs, g_j in grids.values():
            g_gs.u.zero_()
            g_j.u.zero_()
        if ev is not None:
            ev[0].record(stream)
        grids["fd7"][0].gs(SWEEPS, tmp=gs_tmp)
        if ev is not None:
            ev[1].record(stream)
        grids["q1_27"][0].gs(SWEEPS, tmp=gs_tmp)
        if ev is not None:
            ev[2].record(stream)
        grids["fd7"][1].jacobi(OMEGA, SWEEPS, tmp)
        if ev is not None:
            ev[3].record(stream)
        grids["q1_27"][1].jacobi(OMEGA, SWEEPS, tmp)
        if ev is not None:
            ev[4].record(stream)
        grids["fd7"][0].residual(norms=norms[0])
        grids["q1_27"][0].residual(norms=norms[1])
        if ev is not None:
            ev[5].record(stream)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(a.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for s in range(a.steps):
        step(evs[s])
    t_end.record(stream)
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    ms_step = total_ms / a.steps
    row_ms = {r: 0.0 for r in ROWS}
    for s in range(a.steps):
        for i, r in enumerate(ROWS):
            row_ms[r] += evs[s][i].elapsed_time(evs[s][i + 1]) / a.steps

    pts = N ** 3
    updates_per_step = 4 * SWEEPS * pts
    value = updates_per_step / (ms_step * 1e-3) / 1e9
    # sweeps per pass over memory: the library pairs the red-black and the
    # Jacobi sweeps (the intermediate iterate stays on chip), so such a pass
    # moves the 24 bytes per point of one sweep for two updates; the 8-colour
    # sweep is one per pass
    per_pass = {"gs_" + k: (grids[k][0].sweeps_per_pass() if fused_rows[k] else 1) for k in grids}
    per_pass.update({"jacobi_" + k: grids[k][1].sweeps_per_pass(jacobi=True) for k in grids})
    rows = {}
    moved = 0.0
    for r in ROWS[:4]:
        per_sweep_ms = row_ms[r] / SWEEPS
        glups = pts / (per_sweep_ms * 1e-3) / 1e9
        bpu = BYTES_PER_UPDATE / per_pass[r]
        moved += bpu * SWEEPS * pts
        rows[r] = {"ms_per_sweep": round(per_sweep_ms, 5), "GLUP/s": round(glups, 2),
                   "sweeps_per_pass": per_pass[r], "bytes_per_update": bpu,
                   "hbm_frac": round(glups * bpu / HBM_PEAK_GBS, 4),
                   "effective_frac_per_sweep": round(glups * BYTES_PER_UPDATE / HBM_PEAK_GBS, 4)}
    rows["residuals"] = {"ms": round(row_ms["residuals"], 5)}

    # dominant kernel: the sweep row with the largest time
    dom = max(ROWS[:4], key=lambda r: row_ms[r])
    if dom.startswith("gs"):
        st_name = "fd7" if dom == "gs_fd7" else "q1_27"
        fused = fused_rows[st_name]
        if fused and per_pass[dom] == 2:
            kernel = "fused_gs_two_sweeps_" + st_name
            launches = SWEEPS // 2
            bytes_per_launch = BYTES_PER_UPDATE * pts
        elif fused:
            kernel = "fused_gs_sweep_" + st_name
            launches = SWEEPS
            bytes_per_launch = BYTES_PER_UPDATE * pts
        else:
            kernel = "colour_pass_" + st_name
            nc = 2 if st_name == "fd7" else 8
            launches = SWEEPS * nc
            bytes_per_launch = BYTES_PER_UPDATE * pts / nc
    elif per_pass[dom] == 2:
        kernel = "jacobi_two_sweeps_" + dom.split("_", 1)[1]
        launches = SWEEPS // 2
        bytes_per_launch = BYTES_PER_UPDATE * pts
    else:
        kernel = "jacobi_" + dom.split("_", 1)[1]
        launches = SWEEPS
        bytes_per_launch = BYTES_PER_UPDATE * pts
    # the row also holds the halo copy (and the copy back for odd counts); the
    # mean launch duration below charges that to the kernel (conservative)
    mean_launch_s = row_ms[dom] * 1e-3 / launches
    achieved = bytes_per_launch / mean_launch_s / 1e9
    if kernel.startswith("fused"):
        src = ["paper_1810_04033_amd/csrc/k_fused.hip", "paper_1810_04033_amd/csrc/cs_tiles.h",
               "paper_1810_04033_amd/csrc/cs_device.h"]
    elif kernel.startswith("jacobi"):
        src = ["paper_1810_04033_amd/csrc/k_stream.hip", "paper_1810_04033_amd/csrc/cs_device.h"]
    else:
        src = ["paper_1810_04033_amd/csrc/k_basic.hip", "paper_1810_04033_amd/csrc/cs_device.h"]
    sha = _source_sha(src)
    traffic = _traffic(kernel, sha)
    roofline = {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "bytes_per_launch": int(bytes_per_launch),
                "mean_launch_us": round(mean_launch_s * 1e6, 3), "source_sha": sha}

    out = {
        "metric": "GLUP/s (grid-point updates per second over coloured GS and Jacobi sweeps)",
        "value": round(value, 3), "unit": "GLUP/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "3D Poisson 256^3 interior, h=1/257, FP64, zero Dirichlet, "
                               "seeded uniform[-1,1) RHS, u0=0; per step 100 red-black GS sweeps "
                               "(7-point), 100 8-colour GS sweeps (27-point trilinear), 100 "
                               "weighted Jacobi sweeps (omega=2/3) of each stencil, residual norms",
                   "grid": [N, N, N], "sweeps_per_row": SWEEPS,
                   "gs_mode": {k: ("fused single pass" if v else "one launch per colour")
                               for k, v in fused_rows.items()}},
        # hbm_frac: bytes the passes move over the step time (the real share of
        # HBM bandwidth); effective_frac_per_sweep: 24 bytes per update of a
        # single sweep over the time per sweep, which exceeds what HBM could
        # move where sweeps run two per pass
        "hbm_frac": round(moved / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "effective_frac_per_sweep": round(value * BYTES_PER_UPDATE / HBM_PEAK_GBS, 4),
        "rows": rows,
        "roofline": roofline,
        "final_rel_residual": [float(x) for x in (norms[:, 0] / norms[:, 2]).cpu().numpy()],
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
        out["cpu_openmp"] = cpu_baseline(openmp=True)
    if not a.no_growth:
        # the growth rows, bounded: the 4096-patch batch (3 timed runs of 20
        # sweeps against one launch per patch and colour) and a 100-request
        # serving stream; each block is freed before the next
        del grids, tmp, b
        torch.cuda.empty_cache()
        pa = patches_measure(steps=3, warmup=1, tune=False, baselines=("per_colour",))
        out["patches_4096"] = {k: pa[k] for k in ("value", "unit", "ms_per_step", "patches_per_s",
                                                  "speedup_vs_per_patch_launches")}
        out["patches_4096"]["baseline_ms_one_launch_per_patch_per_colour"] = \
            pa["baseline_ms"]["one_launch_per_patch_per_colour"]
        torch.cuda.empty_cache()
        from paper_1810_04033_amd import serve as SV
        sv = SV.serve_measure(100)
        out["serve_100"] = {"patches_per_s": sv["value"],
                            "p50_latency_s": sv["served"]["offered_2000_per_s"]["p50_latency_s"],
                            "p99_latency_s": sv["served"]["offered_2000_per_s"]["p99_latency_s"],
                            "gpu_busy_fraction": sv["served"]["offered_2000_per_s"]["gpu_busy_fraction"],
                            "at_0.8x_capacity": {k: sv["served"]["offered_0.8x_capacity"][k]
                                                 for k in ("rate_per_s", "patches_per_s",
                                                           "p50_latency_s", "p99_latency_s")},
                            "speedup_vs_one_patch_per_launch": sv["speedup_vs_one_patch_per_launch"],
                            "workload": sv["config"]["workload"]}
    print(json.dumps(out), flush=True)


def run_patches(a):
    out = patches_measure(a.steps, a.warmup, a.tune, cpu=not a.no_cpu_baseline,
                          baselines=tuple(m for m in a.patch_baselines.split(",") if m))
    print(json.dumps(out), flush=True)


def patches_measure(steps, warmup, tune, baselines=("per_colour", "fused_per_patch"), cpu=False):
    """4096 cubic patches, edges uniform over {8,16,24,32,48,64} (seed 3), zero
    halo, uniform[-1,1) RHS per patch (stream = patch id), u0 = 0, 20 red-black
    7-point GS sweeps in FP64: the batch (small patches resident in LDS for all
    sweeps, the others one launch per tile group and pass) against one launch
    per patch and colour (and one fused launch per patch and sweep)."""
    import numpy as np
    import torch

    from paper_1810_04033_amd import colsten as C
    from paper_1810_04033_amd import inputs as I
    from paper_1810_04033_amd import tune as TU

    torch.cuda.set_device(0)
    sweeps = 20
    tuned = TU.tune(C.CS_FD, torch.float64) if tune else TU.apply_cached(C.CS_FD, torch.float64)
    edges = I.patch_edges(3, 4096)
    ps = []
    for i, e in enumerate(edges):
        u = C.empty_grid((e, e, e))
        b = C.empty_grid((e, e, e))
        b.copy_(torch.from_numpy(I.halo_array(I.uniform_field(I.stream_seed(3, i), (e, e, e)))))
        ps.append((u, b, C.grid_like(u), C.CS_FD, 1.0 / (e + 1), 0))
    pts = sum(e ** 3 for e in edges)
    bt = C.Batch(ps)
    stream = torch.cuda.current_stream()

    def reset():
        for u, *_ in ps:
            u.zero_()

    for _ in range(warmup):
        reset()
        bt.gs(sweeps)
    times = []
    for _ in range(steps):
        reset()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        bt.gs(sweeps)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = sum(times) / len(times)
    norms = bt.residual().cpu().numpy()
    per_pass = [bt.sweeps_per_pass(i) for i in range(len(ps))]
    bt.close()

    # one launch per patch per colour pass (in place), then one fused launch per sweep
    base = {}
    for mode in baselines:
        reset()
        grids = [C.Grid(u, b, dim=3, stencil=C.CS_FD, h=h) for (u, b, t, st, h, par) in ps]
        for g in grids:
            # the baselines as named: colour passes, or one fused pass per sweep
            # (not the automatic schedules of small grids)
            g.set_pass_mode(C.CS_PASS_ONE)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for g, p in zip(grids, ps):
            g.gs(sweeps, tmp=p[2] if mode == "fused_per_patch" else None)
        e1.record(stream)
        torch.cuda.synchronize()
        base[mode] = e0.elapsed_time(e1)
        for g in grids:
            g.close()

    value = pts * sweeps / (ms * 1e-3) / 1e9
    # bytes moved per sweep: 24 per point and pass over memory, over the
    # sweeps: a patch swept k sweeps per pass makes ceil(sweeps / k) passes
    # (one sweep per pass: 24 B per update; two: 12; streamed three per pass:
    # 24 x 7 / 20), a patch resident in LDS one pass for all sweeps
    passes = [-(-sweeps // k) if k else 1 for k in per_pass]
    bytes_per_sweep = sum(24 * e ** 3 * n / sweeps for e, n in zip(edges, passes))
    paired_pts = sum(e ** 3 for e, k in zip(edges, per_pass) if k == 2)
    achieved = bytes_per_sweep / (ms * 1e-3 / sweeps) / 1e9
    out = {
        "metric": "GLUP/s and patches/s (batched coloured GS on 4096 patches)",
        "value": round(value, 3), "unit": "GLUP/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "4096 cubic patches, edge uniform over {8,16,24,32,48,64} (seed 3), "
                               "FP64 7-point red-black GS, 20 sweeps per patch, zero Dirichlet halo",
                   "points": pts, "sweeps": sweeps, "tile_policy": tuned},
        "patches_per_s": round(4096 / (ms * 1e-3), 1),
        "baseline_ms": {("one_launch_per_patch_per_colour" if m == "per_colour" else
                         "one_fused_launch_per_patch_per_sweep"): round(v, 3) for m, v in base.items()},
        "speedup_vs_per_patch_launches": (round(base["per_colour"] / ms, 2)
                                          if "per_colour" in base else None),
        "roofline": {"bound": "hbm", "kernel": "batched_gs_fd7", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "bytes_per_sweep": int(bytes_per_sweep),
                     "mean_sweep_us": round(ms * 1e3 / sweeps, 3),
                     "points_swept_two_per_pass": paired_pts,
                     "streamed_points": sum(e ** 3 for e, k in zip(edges, per_pass) if k >= 3),
                     "note": "bytes moved per sweep over the time per sweep: 24 B per point and "
                             "pass over memory; patches of the large tile class run two sweeps per "
                             "pass, streamed patches three (the last pass two), patches resident "
                             "in LDS all sweeps in one pass, the others one sweep per pass"},
        "max_final_rel_residual": float(np.max(norms[:, 0] / norms[:, 2])),
    }
    if cpu:
        from oracle import oracle as O
        t0 = time.perf_counter()
        sample_pts = 0
        for i in (0, 1, 2, 3, 4, 5, 6, 7):
            e = edges[i]
            bh = I.halo_array(I.uniform_field(I.stream_seed(3, i), (e, e, e)))
            uo = I.halo_array(np.zeros((e, e, e)))
            O.gs_sweeps(uo, bh, sweeps, dim=3, stencil=O.FD, h=1.0 / (e + 1))
            sample_pts += e ** 3
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": sample_pts * sweeps / dt / 1e9, "unit": "GLUP/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "patches 0-7 of the same set, 20 sweeps each, sequential "
                                         "C oracle, %.1f s" % dt}
    del ps
    return out


def run_refine(a):
    """3D Poisson, n^3 interior (default 512), h = 1/(n+1), 27-point trilinear
    8-colour GS.  RHS: 32 random Fourier modes (frequencies 1..32, N(0,1)
    amplitudes) plus uniform[-1e-3, 1e-3] noise, seed 4.  FP32 sweeps inside
    FP64 iterative refinement to 1e-10 relative residual, against FP64 sweeps
    to the same tolerance; the final residual of each is recomputed by the
    oracle in FP64 on the host."""
    import numpy as np
    import torch

    from paper_1810_04033_amd import colsten as C
    from paper_1810_04033_amd import inputs as I
    from paper_1810_04033_amd import solve as S

    torch.cuda.set_device(0)

    def say(msg):
        print("[refine] " + msg, file=sys.stderr, flush=True)

    last = [0.0]

    def progress(sweeps, rel):
        if time.perf_counter() - last[0] > 20.0:
            last[0] = time.perf_counter()
            say("%d sweeps, relative residual %.3e" % (sweeps, rel))

    n = a.refine_n
    h = 1.0 / (n + 1)
    tol = 1e-10
    inner = 200
    n3 = (n, n, n)
    t0 = time.perf_counter()
    b_host = I.halo_array(I.fourier_field(4, n))
    gen_s = time.perf_counter() - t0
    b = C.empty_grid(n3)
    b.copy_(torch.from_numpy(b_host))
    x = C.empty_grid(n3)
    e = C.empty_grid(n3, dtype=torch.float32)
    r32 = C.empty_grid(n3, dtype=torch.float32)
    tmp32 = C.grid_like(e)
    g64 = C.Grid(x, b, dim=3, stencil=C.CS_Q1, h=h)
    g32 = C.Grid(e, r32, dim=3, stencil=C.CS_Q1, h=h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    say("refinement solve, n = %d" % n)
    ir = S.ir_solve(g64, g32, tol, inner_sweeps=inner, tmp32=tmp32, progress=progress)
    torch.cuda.synchronize()
    ir_s = time.perf_counter() - t0
    x_ir = x.detach().cpu().numpy()
    del e, r32, tmp32
    u = C.empty_grid(n3)
    tmp = C.grid_like(u)
    gp = C.Grid(u, b, dim=3, stencil=C.CS_Q1, h=h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    say("refinement done in %.1f s; FP64 solve" % ir_s)
    fp = S.gs_solve(gp, tol, check_every=inner, tmp=tmp, progress=progress)
    torch.cuda.synchronize()
    fp_s = time.perf_counter() - t0
    out = {
        "metric": "seconds to 1e-10 relative residual (FP32 sweeps in FP64 refinement vs FP64 sweeps)",
        "value": round(ir_s, 3), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(ir_s * 1e3, 1), "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None, "dtype": "f32 sweeps / f64 residual and update", "data": "synthetic",
        "config": {"workload": "3D Poisson %d^3, 27-point trilinear 8-colour GS, Fourier+noise RHS "
                               "(seed 4), tol 1e-10, %d inner FP32 sweeps per refinement step"
                               % (n, inner)},
        "refine": {"seconds": round(ir_s, 3), "outer": ir.outer, "sweeps": ir.sweeps,
                   "rel_residual_gpu": ir.rel_residual, "converged": ir.converged,
                   "GLUP/s": round(n ** 3 * ir.sweeps / ir_s / 1e9, 2)},
        "fp64": {"seconds": round(fp_s, 3), "sweeps": fp.sweeps, "rel_residual_gpu": fp.rel_residual,
                 "converged": fp.converged, "GLUP/s": round(n ** 3 * fp.sweeps / fp_s / 1e9, 2)},
        "speedup": round(fp_s / ir_s, 3), "rhs_generation_s": round(gen_s, 1),
    }
    if not a.no_cpu_baseline:
        from oracle import oracle as O
        say("FP64 done in %.1f s; oracle residual checks" % fp_s)
        t0 = time.perf_counter()
        nr = O.residual(x_ir, b_host, dim=3, stencil=O.Q1, h=h)
        say("oracle check 1 of 2 done")
        out["refine"]["rel_residual_oracle_fp64"] = float(nr[0] / nr[2])
        nf = O.residual(u.detach().cpu().numpy(), b_host, dim=3, stencil=O.Q1, h=h)
        out["fp64"]["rel_residual_oracle_fp64"] = float(nf[0] / nf[2])
        out["oracle_check_s"] = round(time.perf_counter() - t0, 1)
    print(json.dumps(out), flush=True)


def run_multigrid(a):
    """3D Poisson, n^3 interior with n = 2^m - 1 (default 255), h = 1/(n+1),
    uniform[-1,1) right-hand side (seed 2) made on the device, u0 = 0.
    Multigrid V(2,2)-cycles whose smoother is the coloured Gauss-Seidel sweep
    (red-black 7-point, 8-colour 27-point), full weighting and d-linear
    interpolation down to one point, to 1e-10 relative residual; against the
    coloured sweeps alone to the same tolerance.  The final residual of each
    multigrid solve is recomputed by the oracle in FP64 on the host."""
    import numpy as np
    import torch

    from paper_1810_04033_amd import colsten as C
    from paper_1810_04033_amd import mg as MG
    from paper_1810_04033_amd import solve as S

    torch.cuda.set_device(0)

    def say(msg):
        print("[multigrid] " + msg, file=sys.stderr, flush=True)

    last = [0.0]

    def progress(sweeps, rel):
        if time.perf_counter() - last[0] > 20.0:
            last[0] = time.perf_counter()
            say("%d sweeps, relative residual %.3e" % (sweeps, rel))

    n = a.mg_n
    if n < 3 or (n + 1) & n:
        raise SystemExit("--mg-n must be 2^m - 1")
    h = 1.0 / (n + 1)
    tol = 1e-10
    n3 = (n, n, n)
    rows = {}
    for name, st in (("fd7", C.CS_FD), ("q1_27", C.CS_Q1)):
        b = C.empty_grid(n3)
        C.fill_uniform(b, 2, dim=3)
        u = C.empty_grid(n3)
        g = C.Grid(u, b, dim=3, stencil=st, h=h)
        mg = MG.Multigrid(g)
        mg.cycle()  # warm-up (first launches), then start again from zero
        torch.cuda.synchronize()
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = mg.solve(tol, max_cycles=100)
        torch.cuda.synchronize()
        mg_s = time.perf_counter() - t0
        say("%s: %d cycles, %.3f s, relative residual %.3e" % (name, res.outer, mg_s, res.rel_residual))
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            mg.cycle()
        e1.record(stream)
        torch.cuda.synchronize()
        cycle_ms = e0.elapsed_time(e1) / 5
        mg.capture()
        mg.cycle_graph()
        e0.record(stream)
        for _ in range(5):
            mg.cycle_graph()
        e1.record(stream)
        torch.cuda.synchronize()
        cycle_graph_ms = e0.elapsed_time(e1) / 5
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        resg = mg.solve(tol, max_cycles=100, graph=True)
        torch.cuda.synchronize()
        mg_graph_s = time.perf_counter() - t0
        say("%s: captured cycles, %d cycles, %.3f s" % (name, resg.outer, mg_graph_s))
        factors = [res.history[i + 1] / res.history[i] for i in range(1, len(res.history) - 1)]
        row = {"cycles": res.outer, "seconds": round(mg_s, 4), "ms_per_cycle": round(cycle_ms, 3),
               "seconds_graph": round(mg_graph_s, 4), "ms_per_cycle_graph": round(cycle_graph_ms, 3),
               "cycles_graph": resg.outer,
               "levels": mg.depth, "rel_residual_gpu": res.rel_residual, "converged": res.converged,
               "mean_factor_per_cycle": float(np.exp(np.mean(np.log(factors)))) if factors else None}
        if not a.no_cpu_baseline:
            from oracle import oracle as O
            u.zero_()
            res2 = mg.solve(tol, max_cycles=100)
            torch.cuda.synchronize()
            nr = O.residual(u.detach().cpu().numpy(), b.detach().cpu().numpy(), dim=3,
                            stencil=O.FD if st == C.CS_FD else O.Q1, h=h)
            row["rel_residual_oracle_fp64"] = float(nr[0] / nr[2])
            row["oracle_cycles"] = res2.outer
        # the same solve by FP32 V-cycles inside FP64 iterative refinement:
        # 3 FP32 cycles per refinement step on the correction equation
        e32 = C.empty_grid(n3, dtype=torch.float32)
        r32 = C.empty_grid(n3, dtype=torch.float32)
        g32 = C.Grid(e32, r32, dim=3, stencil=st, h=h)
        mg32 = MG.Multigrid(g32)
        per_step = 3

        def inner(s, mg32=mg32):
            for _ in range(per_step):
                mg32.cycle(stream=s)

        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ir = S.ir_solve(g, g32, tol, inner_sweeps=per_step, inner=inner, max_outer=50)
        torch.cuda.synchronize()
        ir_s = time.perf_counter() - t0
        row["fp32_cycles_in_fp64_refinement"] = {
            "seconds": round(ir_s, 4), "refinement_steps": ir.outer, "fp32_cycles": ir.sweeps,
            "rel_residual_gpu": ir.rel_residual, "converged": ir.converged}
        say("%s: FP32 cycles in FP64 refinement, %d steps, %.3f s" % (name, ir.outer, ir_s))
        if not a.no_cpu_baseline:
            nr = O.residual(u.detach().cpu().numpy(), b.detach().cpu().numpy(), dim=3,
                            stencil=O.FD if st == C.CS_FD else O.Q1, h=h)
            row["fp32_cycles_in_fp64_refinement"]["rel_residual_oracle_fp64"] = float(nr[0] / nr[2])
        mg32.close()
        g32.close()
        del e32, r32
        mg.close()
        if a.mg_gs_compare:
            u2 = C.empty_grid(n3)
            tmp = C.grid_like(u2)
            g2 = C.Grid(u2, b, dim=3, stencil=st, h=h)
            torch.cuda.synchronize()
            say("%s: coloured sweeps alone to %.0e" % (name, tol))
            t0 = time.perf_counter()
            gs = S.gs_solve(g2, tol, check_every=1000, tmp=tmp, progress=progress)
            torch.cuda.synchronize()
            gs_s = time.perf_counter() - t0
            row["gs_alone"] = {"seconds": round(gs_s, 3), "sweeps": gs.sweeps,
                               "rel_residual_gpu": gs.rel_residual, "converged": gs.converged}
            row["speedup_vs_gs"] = round(gs_s / mg_s, 1)
            g2.close()
            del u2, tmp
        rows[name] = row
        g.close()
        del u, b
        torch.cuda.empty_cache()
    total = rows["fd7"]["seconds"] + rows["q1_27"]["seconds"]
    out = {
        "metric": "seconds to 1e-10 relative residual, multigrid V(2,2) with the coloured "
                  "Gauss-Seidel smoother (7-point and 27-point solves)",
        "value": round(total, 4), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(total * 1e3, 2), "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "3D Poisson %d^3, h=1/%d, uniform[-1,1) RHS (seed 2), u0=0; V(2,2)-"
                               "cycles, full weighting, d-linear interpolation, %d levels to one "
                               "point, 2 sweeps on the coarsest; tol 1e-10" % (n, n + 1, rows["fd7"]["levels"])},
        "rows": rows,
    }
    print(json.dumps(out), flush=True)


EXPENSIVE_CASES = (
    # name, dim, stencil, interior n (x first), kmax, hetero
    ("fd5_2d_k100", 2, 0, (2048, 2048), 100, 0),
    ("fd5_2d_hetero", 2, 0, (2048, 2048), 100, 1),
    ("q1_27_3d_k100", 3, 1, (128, 128, 128), 100, 0),
    ("q1_27_3d_hetero", 3, 1, (128, 128, 128), 100, 1),
)
FP64_VECTOR_PEAK_TFLOPS = 78.6
VALU_ISSUE_PEAK = 256 * 4 * 16 * 2.4e9  # lane-instructions per second


def _expensive_counts(name, sha):
    """FP64 flops per sweep of one expensive case from the committed rocprofv3
    counter summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "expensive_valu.txt")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except ValueError:
        return None
    rec = data.get(name)
    if not rec or rec.get("source_sha") != sha:
        return None
    return rec


def run_expensive(a):
    """Gauss-Seidel sweeps with the expensive stencil evaluation S(k) (Sec. 2; the
    load patterns of Sec. 4): every nonzero stencil entry costs k evaluations of
    sin, with k = 100 everywhere or k running linearly 0..99 over the mesh.
    2D 5-point on 2048^2 and 3D 27-point on 128^3, FP64, one launch per colour.
    The iterate equals the k = 0 iterate bit for bit (tested)."""
    import numpy as np
    import torch

    from paper_1810_04033_amd import colsten as C
    from paper_1810_04033_amd import inputs as I

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    sweeps = 3
    rows = {}
    total_updates = 0
    total_ms = 0.0
    sha = _source_sha(["paper_1810_04033_amd/csrc/k_basic.hip", "paper_1810_04033_amd/csrc/cs_device.h"])
    for name, dim, st, n, kmax, het in EXPENSIVE_CASES:
        shape = tuple(reversed(n))
        u = C.empty_grid(n)
        b = C.empty_grid(n)
        b.copy_(torch.from_numpy(I.halo_array(I.uniform_field(I.stream_seed(6, len(rows)), shape))))
        g = C.Grid(u, b, dim=dim, stencil=st, h=1.0 / (max(n) + 1))
        for _ in range(a.warmup):
            g.gs_cost(1, kmax, hetero=bool(het))
        torch.cuda.synchronize()
        u.zero_()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(a.steps):
            g.gs_cost(sweeps, kmax, hetero=bool(het))
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / (a.steps * sweeps)
        pts = int(np.prod(n))
        entries = (5 if st == 0 else 9) if dim == 2 else (7 if st == 0 else 21)
        # sin evaluations per sweep: entries * sum over points of k(l)
        if het:
            ks = (kmax * np.arange(pts, dtype=np.int64)) // pts
            sins = entries * int(ks.sum())
        else:
            sins = entries * kmax * pts
        rec = _expensive_counts(name, sha)
        rows[name] = {"grid": list(n), "stencil": ["fd", "q1"][st], "kmax": kmax, "hetero": bool(het),
                      "ms_per_sweep": round(ms, 4), "GLUP/s": round(pts / ms / 1e6, 4),
                      "Gsin/s": round(sins / ms / 1e6, 1),
                      "fp64_TFLOP/s": None if rec is None else round(rec["fp64_flops_per_sweep"] / ms / 1e9, 2),
                      "valu_issue_frac": None if rec is None else
                      round(rec["valu_lane_instr_per_sweep"] / (ms * 1e-3) / VALU_ISSUE_PEAK, 4)}
        total_updates += pts
        total_ms += ms
        g.close()
        del u, b
    dom = max(rows, key=lambda r: rows[r]["ms_per_sweep"])
    achieved = rows[dom]["fp64_TFLOP/s"]
    out = {
        "metric": "GLUP/s (coloured GS with the expensive stencil evaluation S(k))",
        "value": round(total_updates / total_ms / 1e6, 4), "unit": "GLUP/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(total_ms * sweeps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "S(k) sweeps: each nonzero stencil entry recomputed with k sin "
                               "evaluations adding exact zeros; 2D 5-point 2048^2 and 3D 27-point "
                               "128^3, k = 100 or k linear 0..99 over the mesh, FP64, %d sweeps "
                               "per case per step" % sweeps},
        "rows": rows,
        "roofline": {"bound": "alu", "kernel": "colour_pass_cost_" + dom,
                     "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": None if achieved is None else round(achieved / FP64_VECTOR_PEAK_TFLOPS, 4),
                     "traffic": None, "valu_issue_frac": rows[dom]["valu_issue_frac"],
                     "source_sha": sha,
                     "note": "FP64 flops and VALU lane-instructions per sweep from rocprofv3 "
                             "SQ_INSTS_VALU* counters (profiles/expensive_valu.txt) over the live "
                             "sweep time; VALU issue peak 256 CU x 4 SIMD x 16 lanes x 2.4 GHz"},
    }
    if not a.no_cpu_baseline:
        from oracle import oracle as O
        n = (2048, 256)
        shape = tuple(reversed(n))
        bh = I.halo_array(I.uniform_field(I.stream_seed(6, 0), shape))
        uo = I.halo_array(np.zeros(shape))
        t0 = time.perf_counter()
        O.gs_sweeps_cost(uo, bh, 1, 100, 0, dim=2, stencil=O.FD, h=1.0 / 2049)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 2048 * 256 / dt / 1e9, "unit": "GLUP/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "one S(k) sweep, k = 100, 2D 5-point on 2048 x 256 (1/8 of "
                                         "the fd5_2d_k100 grid), sequential C oracle, %.1f s" % dt}
    print(json.dumps(out), flush=True)


ORDERING_CASES = (
    # name, dim, stencil, interior n (x first)
    ("fd5_2d_256", 2, 0, (256, 256)),
    ("q1_9_2d_256", 2, 1, (256, 256)),
    ("fd7_3d_128", 3, 0, (128, 128, 128)),
    ("q1_27_3d_128", 3, 1, (128, 128, 128)),
)


def run_orderings(a):
    """Lexicographic Gauss-Seidel (the task-graph iterate of Sec. 3, run as
    hyperplane wavefronts, one launch per hyperplane) and nested-dissection
    Gauss-Seidel (the other ordering of Sec. 3, one launch per tree height,
    leaves of edge 16) beside the coloured sweeps
    (one launch per colour, one persistent launch with a device-wide barrier per
    colour, one persistent launch with tile dependencies, and the fused single
    pass where it exists), FP64,
    on the 2D 256^2 grid of the small workload and a 3D 128^3 grid; the
    launch-per-kernel modes also as captured HIP graphs of 5 sweeps."""
    import numpy as np
    import torch

    from paper_1810_04033_amd import colsten as C
    from paper_1810_04033_amd import inputs as I

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    sweeps = 5
    rows = {}
    lex_ms = lex_pts = 0.0
    for idx, (name, dim, st, n) in enumerate(ORDERING_CASES):
        shape = tuple(reversed(n))
        u = C.empty_grid(n)
        b = C.empty_grid(n)
        b.copy_(torch.from_numpy(I.halo_array(I.uniform_field(I.stream_seed(7, idx), shape))))
        tmp = C.grid_like(u)
        g = C.Grid(u, b, dim=dim, stencil=st, h=1.0 / (max(n) + 1))
        graphs = {"lexicographic_wavefront_graph": C.Graph.of_grid(g, sweeps, lexicographic=True),
                  "coloured_per_colour_graph": C.Graph.of_grid(g, sweeps)}
        modes = {"lexicographic_wavefront": lambda k: g.gs_lex(k),
                 "lexicographic_wavefront_graph": lambda k: [graphs["lexicographic_wavefront_graph"].launch()
                                                             for _ in range(k // sweeps)],
                 "coloured_per_colour": lambda k: g.gs(k),
                 "coloured_persistent_barrier": lambda k: g.gs_sync(k),
                 "coloured_tile_dependencies": lambda k: g.gs_dep(k),
                 "nested_dissection": lambda k: g.gs_nd(k, leaf=16),
                 "coloured_per_colour_graph": lambda k: [graphs["coloured_per_colour_graph"].launch()
                                                         for _ in range(k // sweeps)]}
        if g.fused:
            modes["coloured_fused"] = lambda k: g.gs(k, tmp=tmp)
        pts = int(np.prod(n))
        row = {"grid": list(n)}
        for mode, fn in modes.items():
            fn(sweeps * max(a.warmup, 1))
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(a.steps):
                fn(sweeps)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / (a.steps * sweeps)
            row[mode] = {"ms_per_sweep": round(ms, 4), "GLUP/s": round(pts / ms / 1e6, 3)}
            if mode in ("coloured_persistent_barrier", "coloured_tile_dependencies"):
                row[mode]["waits_given_up"] = g.sync_failures()
            if mode == "lexicographic_wavefront":
                lex_ms += ms
                lex_pts += pts
        wj, wk = (1, 1) if st == 0 else (2, 4)
        row["launches_per_sweep_lexicographic"] = n[0] + wj * n[1] + (wk * n[2] if dim == 3 else 0) - (
            wj + (wk if dim == 3 else 0))
        rows[name] = row
        for gr in graphs.values():
            gr.close()
        g.close()
        del u, b, tmp
    out = {
        "metric": "GLUP/s (lexicographic Gauss-Seidel by hyperplane wavefronts)",
        "value": round(lex_pts / lex_ms / 1e6, 4), "unit": "GLUP/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(lex_ms * sweeps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "lexicographic GS (one launch per hyperplane) against coloured GS "
                               "on 2D 256^2 and 3D 128^3, both stencils, FP64, %d sweeps per mode "
                               "per step" % sweeps},
        "rows": rows,
    }
    if not a.no_cpu_baseline:
        from oracle import oracle as O
        n = (128, 128, 16)
        shape = tuple(reversed(n))
        bh = I.halo_array(I.uniform_field(I.stream_seed(7, 2), shape))
        uo = I.halo_array(np.zeros(shape))
        t0 = time.perf_counter()
        O.lex_sweeps(uo, bh, 5, dim=3, stencil=O.FD, h=1.0 / 129)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 5 * int(np.prod(n)) / dt / 1e9, "unit": "GLUP/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "5 lexicographic 7-point sweeps on 128 x 128 x 16, sequential "
                                         "C oracle, %.2f s" % dt}
    print(json.dumps(out), flush=True)


XGMI_LINK_GBS = 153.0  # one xGMI link, per direction


def run_slab(a):
    """One GPU's share of a grid cut into z-slabs: the four sweep rows of the
    headline step on each slab shape (100 sweeps each, FP64 by default, the
    slab's halo standing in for its neighbours' planes), beside the time a
    one-link exchange of the planes the next pass needs would take (2 planes
    per side per sweep, each way).  The shapes, element type, rows and sweep
    count are options, so the same rows can be timed (and profiled) on a whole
    grid such as 512^3."""
    import torch

    from paper_1810_04033_amd import colsten as C

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    shapes = [tuple(int(v) for v in s.split(",")) for s in a.slab.split(";")]
    for n in shapes:
        if len(n) != 3 or min(n) < 1:
            raise SystemExit("--slab: shapes are nx,ny,nz;...")
    dt = torch.float64 if a.slab_dtype == "f64" else torch.float32
    want = set(a.slab_rows.split(","))
    nsw = a.slab_sweeps
    res = {}
    for n in shapes:
        pts = n[0] * n[1] * n[2]
        b = C.empty_grid(n, dtype=dt)
        C.fill_uniform(b, 2, dim=3)
        tmp = C.empty_grid(n, dtype=dt)
        h = 1.0 / (max(n) + 1)
        rows = {}
        for name, st in (("fd7", C.CS_FD), ("q1_27", C.CS_Q1)):
            if not any(k + "_" + name in want for k in ("gs", "jacobi")):
                continue
            u = C.empty_grid(n, dtype=dt)
            g = C.Grid(u, b, dim=3, stencil=st, h=h)
            for kind in ("gs", "jacobi"):
                if kind + "_" + name not in want:
                    continue

                def run():
                    u.zero_()
                    e0.record(stream)
                    if kind == "gs":
                        g.gs(nsw, tmp=tmp)
                    else:
                        g.jacobi(OMEGA, nsw, tmp)
                    e1.record(stream)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                for _ in range(a.warmup):
                    run()
                torch.cuda.synchronize()
                ms = 0.0
                for _ in range(a.steps):
                    run()
                    torch.cuda.synchronize()
                    ms += e0.elapsed_time(e1)
                per_sweep_us = ms / a.steps / nsw * 1e3
                rows[kind + "_" + name] = {"us_per_sweep": round(per_sweep_us, 3),
                                           "GLUP/s": round(pts / (per_sweep_us * 1e-6) / 1e9, 2),
                                           "sweeps_per_pass": g.sweeps_per_pass(jacobi=(kind == "jacobi"))}
            g.close()
        exch_bytes = 2 * n[0] * n[1] * (8 if dt == torch.float64 else 4)  # per neighbour, sweep, way
        res["x".join(map(str, n))] = {
            "rows": rows,
            "exchange_bytes_per_neighbour_per_sweep": exch_bytes,
            "exchange_us_per_sweep_one_link": round(exch_bytes / (XGMI_LINK_GBS * 1e9) * 1e6, 3)}
    total = sum(len(v["rows"]) for v in res.values())
    mean = sum(r["GLUP/s"] for v in res.values() for r in v["rows"].values()) / total
    print(json.dumps({
        "metric": "GLUP/s on one GPU's z-slab (mean over the four sweep rows and the shapes)",
        "value": round(mean, 3), "unit": "GLUP/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": a.slab_dtype, "data": "synthetic",
        "config": {"workload": "one GPU's z-slab of a larger 3D Poisson grid (or a whole grid), "
                               "%s, seeded uniform[-1,1) RHS, u0=0, %d sweeps per row"
                               % (a.slab_dtype.upper(), nsw),
                   "slabs": list(res), "rows": sorted(want)},
        "slabs": res}), flush=True)


def run_serve(a):
    from paper_1810_04033_amd import serve as SV
    SV.bench_main(a)


def run_calib(a):
    """A plain device copy of known size for calibrating rocprofv3's byte
    counters: three copies of exactly 1 GiB (2^27 doubles) between two device
    buffers.  The FETCH_SIZE / WRITE_SIZE readings of these dispatches divided
    by 1 GiB are the scale factors applied to the kernels' counter readings."""
    import torch

    torch.cuda.set_device(0)
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"workload": "calib", "copies": 3, "bytes_per_copy": 1 << 30}), flush=True)


def main():
    a = _args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the coloured-sweep path is single-GPU "
              "(see the sharding design); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if a.workload == "patches":
        run_patches(a)
    elif a.workload == "refine":
        run_refine(a)
    elif a.workload == "multigrid":
        run_multigrid(a)
    elif a.workload == "serve":
        run_serve(a)
    elif a.workload == "expensive":
        run_expensive(a)
    elif a.workload == "orderings":
        run_orderings(a)
    elif a.workload == "slab":
        run_slab(a)
    elif a.workload == "calib":
        run_calib(a)
    else:
        run_poisson3d(a)


if __name__ == "__main__":
    main()
