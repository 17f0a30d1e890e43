"""Continuous-batching request server for patch solves.

Requests (3D patch, stencil, precision, right-hand side) arrive over time.
The scheduler admits a waiting request as soon as a slot and enough of the HBM
budget are free, keeps its state resident on the device, and advances all
active requests together in steps: one step runs `sweeps_per_step` coloured
Gauss-Seidel sweeps of every active patch in the same batched launches (the
refinement requests' FP64 residual and correction in one batched launch
each), then copies every patch's residual norms to the host asynchronously.
The GPU executor reads a step's norms while the next step runs (lag 1): a
request whose relative residual reached the tolerance retires one step after
the step that reached it (latency = retirement - arrival), having run that one
more step; its memory is released and waiting requests are admitted at the
next step.

Each request's sweeps happen in steps of fixed size regardless of what else
is active, retirement always lags by the same one step, and the batched
kernels compute every patch independently, so a request's result is the same
alone and in any mix.

The scheduler is independent of the executor: `GpuExecutor` drives libcolsten;
tests drive the scheduler logic with a CPU stand-in executor.
"""
import math
import time
from dataclasses import dataclass, field

import numpy as np

from .solve import pow2_at_least

DONE, DIVERGED, NOT_CONVERGED, REJECTED, CANCELLED = "done", "diverged", "not_converged", "rejected", "cancelled"


@dataclass
class Ticket:
    req: object                 # inputs.Request-like: rid, arrival_s, n, stencil, mixed, rhs_seed
    rhs: object = None          # host interior RHS (nz, ny, nx) float64
    status: str = "waiting"
    admitted_s: float = float("nan")
    finished_s: float = float("nan")
    sweeps: int = 0
    rel_residual: float = float("nan")
    state: object = None
    cancel: bool = False
    result: object = None       # final iterate (host), when the executor keeps results

    @property
    def latency_s(self):
        return self.finished_s - self.req.arrival_s


@dataclass
class ServeStats:
    completed: int = 0
    failed: int = 0
    steps: int = 0
    max_active: int = 0
    peak_bytes: int = 0
    busy_s: float = 0.0         # host time inside executor steps
    gpu_busy_s: float = 0.0     # device time of the steps' work (when the executor times it)
    latencies: list = field(default_factory=list)

    def summary(self, t_first_arrival, t_last_done):
        lat = np.array(self.latencies) if self.latencies else np.array([float("nan")])
        span = max(t_last_done - t_first_arrival, 1e-12)
        return {"completed": self.completed, "failed": self.failed, "steps": self.steps,
                "patches_per_s": self.completed / span,
                "p50_latency_s": float(np.percentile(lat, 50)),
                "p99_latency_s": float(np.percentile(lat, 99)),
                "mean_latency_s": float(np.mean(lat)), "max_active": self.max_active,
                "peak_bytes": self.peak_bytes, "span_s": span,
                "gpu_busy_fraction": self.gpu_busy_s / span if self.gpu_busy_s > 0 else None}


class Scheduler:
    """Admission by slots and memory, stepping, retirement, latency accounting.

    executor must provide: bytes_needed(req), admit(ticket), step(tickets, k)
    -> list of (rel_residual) per ticket, release(ticket).
    clock: callable returning seconds since the start of the run."""

    def __init__(self, executor, *, budget_bytes, max_active=256, sweeps_per_step=50, tol=1e-8,
                 max_sweeps=10 ** 6, clock=None):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.k = int(sweeps_per_step)
        self.tol = float(tol)
        self.max_sweeps = int(max_sweeps)
        self.clock = clock
        self.waiting = []
        self.active = []
        self.finished = []
        self.used = 0
        self.stats = ServeStats()

    def submit(self, ticket):
        need = self.ex.bytes_needed(ticket.req)
        if need > self.budget:
            ticket.status = REJECTED
            ticket.finished_s = ticket.req.arrival_s
            self.finished.append(ticket)
            self.stats.failed += 1
            return
        self.waiting.append(ticket)

    def _admit(self, now):
        # FIFO: the head waits until it fits (no overtaking by smaller requests)
        while self.waiting and len(self.active) < self.max_active:
            t = self.waiting[0]
            if t.req.arrival_s > now:
                break
            if t.cancel:
                self.waiting.pop(0)
                t.status = CANCELLED
                t.finished_s = now
                self.finished.append(t)
                self.stats.failed += 1
                continue
            need = self.ex.bytes_needed(t.req)
            if self.used + need > self.budget:
                break
            self.waiting.pop(0)
            self.used += need
            t.status = "active"
            t.admitted_s = now
            self.ex.admit(t)
            self.active.append(t)
        self.stats.max_active = max(self.stats.max_active, len(self.active))
        self.stats.peak_bytes = max(self.stats.peak_bytes, self.used)

    def _retire(self, t, status, now):
        t.status = status
        t.finished_s = now
        self.used -= self.ex.bytes_needed(t.req)
        self.ex.release(t)
        self.active.remove(t)
        self.finished.append(t)
        if status == DONE:
            self.stats.completed += 1
            self.stats.latencies.append(t.latency_s)
        else:
            self.stats.failed += 1

    def step(self):
        """One scheduler step; returns False when nothing is left to do."""
        now = self.clock()
        self._admit(now)
        for t in [t for t in self.active if t.cancel]:
            self._retire(t, CANCELLED, now)
        lag = getattr(self.ex, "lag", 0)
        if not self.active:
            if lag and self.ex.pending():
                self._results(self.ex.drain(), self.clock())
                return True
            if not self.waiting:
                return False
            # idle until the next arrival
            nxt = self.waiting[0].req.arrival_s
            while self.clock() < nxt:
                time.sleep(min(1e-4, max(0.0, nxt - self.clock())))
            return True
        t0 = self.clock()
        out = self.ex.step(self.active, self.k)
        now = self.clock()
        self.stats.busy_s += now - t0
        self.stats.steps += 1
        # an executor with lag 1 returns the residuals of the step before the
        # one it just enqueued, as (ticket, rel) pairs
        self._results(out if lag else list(zip(list(self.active), out)), now)
        return True

    def _results(self, pairs, now):
        active = set(id(t) for t in self.active)
        for t, rel in pairs:
            if id(t) not in active:
                continue  # retired or cancelled since that step was enqueued
            t.rel_residual = rel
            if not math.isfinite(rel):
                self._retire(t, DIVERGED, now)
            elif rel <= self.tol:
                self._retire(t, DONE, now)
            elif t.sweeps >= self.max_sweeps:
                self._retire(t, NOT_CONVERGED, now)

    def run(self, tickets):
        for t in tickets:
            self.submit(t)
        while self.step():
            pass
        self.stats.gpu_busy_s = getattr(self.ex, "gpu_ms", 0.0) * 1e-3
        return self.finished


class GpuExecutor:
    """Runs admitted requests on the GPU through libcolsten.

    Four reserved batches hold the active patches, one per stencil and
    precision: for FP64 requests u, b and a work array; for refinement
    requests the FP32 correction e, its scaled right-hand side r32 and a work
    array, paired with their FP64 iterate x and right-hand side b.  Each
    request keeps one norm row (its slot) for its life, so a change of the
    active set only reassigns the batches: their tables go to the device by
    asynchronous copies from pinned staging buffers, with no allocation and no
    synchronisation.  A step forks the four batches onto their own streams
    (they share nothing within a step, so steps with few patches still fill
    the device): for refinement requests the batched correction x += s e, the
    batched FP64 residual (scale and FP32 copy on the device) and the sweeps;
    for FP64 requests the sweeps and the batched residual.  It joins them,
    copies all norms to pinned host memory asynchronously, and then waits for
    the previous step's norms, which arrived while this step was queued
    (lag 1)."""

    lag = 1
    LANES = ((False, 0), (False, 1), (True, 0), (True, 1))  # (refinement, stencil)

    def __init__(self, stream=None, keep_results=False, max_active=256, max_edge=128):
        import torch
        from . import colsten as C
        self.torch = torch
        self.C = C
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        # lane 0 runs on the executor's stream, the others on streams of their
        # own (default priority)
        self.streams = [self.stream] + [torch.cuda.Stream(device=self.stream.device)
                                        for _ in self.LANES[1:]]
        self.keep_results = keep_results
        self.max_active = int(max_active)
        self.max_edge = int(max_edge)
        dev = torch.device("cuda", torch.cuda.current_device())
        partials = self.max_active * C.residual_items((max_edge, max_edge, max_edge))
        self.batches = [C.cs_batch_reserve(self.max_active, partials) for _ in self.LANES]
        self.busy = [False] * len(self.LANES)
        self.norms = torch.zeros(self.max_active, 3, dtype=torch.float64, device=dev)
        self.scales = torch.ones(self.max_active, dtype=torch.float64, device=dev)
        self.host = [torch.zeros(self.max_active, 3, dtype=torch.float64).pin_memory() for _ in range(2)]
        self.buf = 0
        self.free_rows = list(range(self.max_active - 1, -1, -1))
        self.dirty = True
        self._pending = None
        self.point_sweeps = 0  # interior points times sweeps, over all steps

    def close(self):
        for i, h in enumerate(getattr(self, "batches", [])):
            if h:
                self.C.cs_batch_destroy(h)
                self.batches[i] = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def bytes_needed(req):
        nx, ny, nz = req.n
        pts = (nx + 2) * (ny + 2) * (nz + 2)
        return pts * (8 * 2 + 4 * 3 if req.mixed else 8 * 3)

    def admit(self, t):
        torch, C = self.torch, self.C
        nx, ny, nz = t.req.n
        if max(t.req.n) > self.max_edge:
            raise ValueError("request edge %d beyond the executor's %d" % (max(t.req.n), self.max_edge))
        n = (nx, ny, nz)
        h = 1.0 / (max(n) + 1)
        with torch.cuda.stream(self.stream):
            b = C.empty_grid(n)
            rhs = torch.from_numpy(t.rhs).pin_memory()
            b[1:-1, 1:-1, 1:nx + 1].copy_(rhs, non_blocking=True)
            u = C.empty_grid(n)
            st = {"h": h, "u": u, "b": b, "row": self.free_rows.pop()}
            if t.req.mixed:
                e = C.empty_grid(n, dtype=torch.float32)
                st.update(e=e, r32=C.empty_grid(n, dtype=torch.float32), tmp=C.grid_like(e))
                # the first scale comes from max |r_0| = max |b| (x = 0)
                self.norms[st["row"], 1].fill_(float(np.max(np.abs(t.rhs))))
            else:
                st["tmp"] = C.grid_like(u)
        t.state = st
        self.dirty = True

    def release(self, t):
        st = t.state
        if st is not None:
            if self.keep_results:
                with self.torch.cuda.stream(self.stream):
                    t.result = st["u"].detach().cpu().numpy()
            self.free_rows.append(st["row"])
        t.state = None
        self.dirty = True

    def _assign(self, tickets):
        C = self.C
        for li, (mixed, stencil) in enumerate(self.LANES):
            ts = [t for t in tickets if t.req.mixed == mixed and t.req.stencil == stencil]
            it, rt = ("e", "r32") if mixed else ("u", "b")
            C.cs_batch_assign(self.batches[li],
                              [C.describe(t.state[it], dim=3, stencil=stencil, h=t.state["h"]) for t in ts],
                              [t.state[it].data_ptr() for t in ts], [t.state[rt].data_ptr() for t in ts],
                              [t.state["tmp"].data_ptr() for t in ts], [t.state["row"] for t in ts],
                              self.stream)
            if mixed:
                C.cs_batch_ir_attach(self.batches[li],
                                     [C.describe(t.state["u"], dim=3, stencil=stencil, h=t.state["h"])
                                      for t in ts],
                                     [t.state["u"].data_ptr() for t in ts],
                                     [t.state["b"].data_ptr() for t in ts], self.stream)
            self.busy[li] = bool(ts)
        self.dirty = False

    def step(self, tickets, k):
        torch, C = self.torch, self.C
        if self.dirty:
            self._assign(tickets)
        s = self.stream
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        fork = torch.cuda.Event()
        fork.record(s)
        joins = []
        for li, (mixed, _) in enumerate(self.LANES):
            if not self.busy[li]:
                continue
            ls, bt = self.streams[li], self.batches[li]
            if ls is not s:
                ls.wait_event(fork)
            if mixed:
                C.cs_batch_ir_update(bt, self.scales.data_ptr(), ls)
                C.cs_batch_ir_residual(bt, self.scales.data_ptr(), self.norms.data_ptr(), ls)
                C.cs_batch_gs_sweeps(bt, k, ls)
            else:
                C.cs_batch_gs_sweeps(bt, k, ls)
                C.cs_batch_residual(bt, self.norms.data_ptr(), ls)
            if ls is not s:
                ev = torch.cuda.Event()
                ev.record(ls)
                joins.append(ev)
        for ev in joins:
            s.wait_event(ev)
        with torch.cuda.stream(s):
            self.host[self.buf].copy_(self.norms, non_blocking=True)
        e1.record(s)
        for t in tickets:
            t.sweeps += k
            nx, ny, nz = t.req.n
            self.point_sweeps += nx * ny * nz * k
        prev = self._pending
        self._pending = ([(t, t.state["row"]) for t in tickets], self.buf, e0, e1)
        self.buf ^= 1
        return self._collect(prev)

    def pending(self):
        return self._pending is not None

    def drain(self):
        prev, self._pending = self._pending, None
        return self._collect(prev)

    def _collect(self, prev):
        if prev is None:
            return []
        pairs, buf, e0, e1 = prev
        e1.synchronize()
        self.gpu_ms = getattr(self, "gpu_ms", 0.0) + e0.elapsed_time(e1)
        host = self.host[buf].numpy()
        out = []
        for t, row in pairs:
            nr = host[row]
            out.append((t, float(nr[0] / nr[2] if nr[2] > 0 else nr[0])))
        return out

    def result(self, t):
        return t.state["u"].detach().cpu().numpy()


def make_tickets(reqs):
    from . import inputs as I
    out = []
    for r in reqs:
        nx, ny, nz = r.n
        out.append(Ticket(r, I.uniform_field(r.rhs_seed, (nz, ny, nx))))
    return out


def bench_main(a):
    """Serving benchmark: see serve_measure; prints one JSON line."""
    import json
    print(json.dumps(serve_measure(int(getattr(a, "serve_count", 0) or 300))), flush=True)


def serve_measure(count):
    """Poisson arrivals of `count` 3D patch solves (edges log-uniform in
    [16, 128], aspect <= 4, 7/27-point and FP64/refinement 50/50, tol 1e-8),
    admitted by a 32 GiB HBM budget and 256 slots: at 2000 requests/s, at 0.8
    times the capacity that run measured, and the same requests one patch per
    launch in FP64."""
    import torch
    from . import colsten as C
    from . import inputs as I
    from . import solve as S

    torch.cuda.set_device(0)
    k = 50
    results = {}

    def serve_at(rate):
        reqs = I.request_stream(5, count, rate)
        tickets = make_tickets(reqs)
        t_start = time.perf_counter()
        clock = lambda: time.perf_counter() - t_start  # noqa: E731
        ex = GpuExecutor(max_active=256)
        sch = Scheduler(ex, budget_bytes=32 << 30, max_active=256, sweeps_per_step=k,
                        tol=1e-8, clock=clock)
        done = sch.run(tickets)
        ex.close()
        t_last = max(t.finished_s for t in done)
        out = sch.stats.summary(reqs[0].arrival_s, t_last)
        # sweep work done per second of the serving span (GS updates / s)
        out["GLUP_per_s"] = ex.point_sweeps / out["span_s"] / 1e9 if out["span_s"] else None
        return out

    # warm-up: a short stream first, as on a server that is already running
    # (first-use costs of the allocator, pinned buffers and kernels)
    reqs = I.request_stream(6, 24, 2000.0)
    ex = GpuExecutor(max_active=256)
    Scheduler(ex, budget_bytes=32 << 30, max_active=256, sweeps_per_step=k, tol=1e-8,
              clock=time.perf_counter).run(make_tickets(reqs))
    ex.close()
    results["offered_2000_per_s"] = serve_at(2000.0)
    capacity = results["offered_2000_per_s"]["patches_per_s"]
    # below capacity the latencies measure service, not queueing
    results["offered_0.8x_capacity"] = serve_at(0.8 * capacity)
    results["offered_0.8x_capacity"]["rate_per_s"] = 0.8 * capacity
    # the same request set one patch per launch in FP64 (colour passes), sequentially
    reqs = I.request_stream(5, count, 2000.0)
    tickets = make_tickets(reqs)
    t0 = time.perf_counter()
    sweeps_seq = 0
    for t in tickets:
        nx, ny, nz = t.req.n
        n = (nx, ny, nz)
        h = 1.0 / (max(n) + 1)
        u = C.empty_grid(n)
        b = C.empty_grid(n)
        b[1:-1, 1:-1, 1:nx + 1].copy_(torch.from_numpy(t.rhs))
        g = C.Grid(u, b, dim=3, stencil=t.req.stencil, h=h)
        g.set_pass_mode(C.CS_PASS_ONE)  # colour passes, as named (not the small-grid schedules)
        r = S.gs_solve(g, 1e-8, check_every=k)
        sweeps_seq += r.sweeps
        g.close()
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t0
    out = {
        "metric": "served patches/s with p50/p99 latency (continuous batching)",
        "value": round(results["offered_2000_per_s"]["patches_per_s"], 2), "unit": "patches/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64 / f32-in-f64 refinement",
        "data": "synthetic",
        "config": {"workload": "%d Poisson arrivals of 3D patch solves at 2000/s, edges log-uniform "
                               "[16,128], aspect <= 4, 7/27-point 50/50, FP64 or FP32-in-FP64 "
                               "refinement 50/50, tol 1e-8, budget 32 GiB, 256 slots, %d sweeps "
                               "per step" % (count, k)},
        "served": results,
        "one_patch_per_launch_fp64": {"seconds": round(seq_s, 3),
                                      "patches_per_s": round(count / seq_s, 2),
                                      "sweeps": sweeps_seq},
        "speedup_vs_one_patch_per_launch": round(results["offered_2000_per_s"]["patches_per_s"]
                                                  / (count / seq_s), 2),
    }
    return out
