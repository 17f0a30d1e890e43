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
    p.add_argument("--per-colour", action="store_true",
                   help="run the GS rows as one launch per colour pass (no work array)")
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
    path = os.path.join(ROOT, "profiles", "traffic.json")
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


def cpu_baseline():
    """The oracle on the host: one sweep of each kind plus both residuals at
    the full 256^3 size (single thread)."""
    import numpy as np
    from oracle import oracle as O
    from paper_1810_04033_amd import inputs as I

    b = I.halo_array(I.uniform_field(2, (N, N, N)))
    t0 = time.perf_counter()
    for st in (O.FD, O.Q1):
        u = I.halo_array(np.zeros((N, N, N)))
        O.gs_sweeps(u, b, 1, dim=3, stencil=st, h=H)
        O.residual(u, b, dim=3, stencil=st, h=H)
        uj = I.halo_array(np.zeros((N, N, N)))
        O.jacobi_sweeps(uj, b, 1, OMEGA, dim=3, stencil=st, h=H)
    dt = time.perf_counter() - t0
    return {"value": 4 * N ** 3 / dt / 1e9, "unit": "GLUP/s", "cores": 1, "kind": "oracle",
            "sample": "one sweep of each of the four sweep kinds plus both residual norms on the "
                      "full 256^3 grid, sequential C oracle, %.1f s" % dt}


def main():
    a = _args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the coloured-sweep path is single-GPU "
              "(see the sharding design); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
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
    rows = {}
    for r in ROWS[:4]:
        per_sweep_ms = row_ms[r] / SWEEPS
        glups = pts / (per_sweep_ms * 1e-3) / 1e9
        rows[r] = {"ms_per_sweep": round(per_sweep_ms, 5), "GLUP/s": round(glups, 2),
                   "hbm_frac_algorithmic": round(glups * BYTES_PER_UPDATE / HBM_PEAK_GBS, 4)}
    rows["residuals"] = {"ms": round(row_ms["residuals"], 5)}

    # dominant kernel: the sweep row with the largest time
    dom = max(ROWS[:4], key=lambda r: row_ms[r])
    if dom.startswith("gs"):
        st_name = "fd7" if dom == "gs_fd7" else "q1_27"
        fused = fused_rows[st_name]
        if fused:
            kernel = "fused_gs_sweep_" + st_name
            launches = SWEEPS
            bytes_per_launch = BYTES_PER_UPDATE * pts
        else:
            kernel = "colour_pass_" + st_name
            nc = 2 if st_name == "fd7" else 8
            launches = SWEEPS * nc
            bytes_per_launch = BYTES_PER_UPDATE * pts / nc
    else:
        kernel = "jacobi_" + dom.split("_", 1)[1]
        launches = SWEEPS
        bytes_per_launch = BYTES_PER_UPDATE * pts
    # the row also holds the halo copy (and the copy back for odd counts); the
    # mean launch duration below charges that to the kernel (conservative)
    mean_launch_s = row_ms[dom] * 1e-3 / launches
    achieved = bytes_per_launch / mean_launch_s / 1e9
    if kernel.startswith("fused"):
        src = ["paper_1810_04033_amd/csrc/k_fused.hip", "paper_1810_04033_amd/csrc/cs_device.h"]
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
        "hbm_frac": round(value * BYTES_PER_UPDATE / HBM_PEAK_GBS, 4),
        "rows": rows,
        "roofline": roofline,
        "final_rel_residual": [float(x) for x in (norms[:, 0] / norms[:, 2]).cpu().numpy()],
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
