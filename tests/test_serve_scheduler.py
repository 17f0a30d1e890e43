"""Scheduler logic of the request server, on the CPU with a stand-in executor:
admission by memory and slots, FIFO order, retirement, latency accounting and
the failure states."""
import math

import numpy as np

from paper_1810_04033_amd import inputs as I
from paper_1810_04033_amd import serve as SV

from fake_executor import FakeExecutor


class Clock:
    """Deterministic clock: advances by `dt` each time it is read."""

    def __init__(self, dt=1e-3):
        self.t = 0.0
        self.dt = dt

    def __call__(self):
        self.t += self.dt
        return self.t


def _req(rid, n, arrival=0.0, stencil=0):
    return I.Request(rid, arrival, n, stencil, False, I.stream_seed(9, rid))


def _tickets(reqs, nan_rid=None):
    out = []
    for r in reqs:
        nx, ny, nz = r.n
        rhs = I.uniform_field(r.rhs_seed, (nz, ny, nx))
        if r.rid == nan_rid:
            rhs[0, 0, 0] = float("nan")
        out.append(SV.Ticket(r, rhs))
    return out


def test_all_requests_complete_and_converge():
    reqs = [_req(i, (4 + i % 3, 5, 4), arrival=0.001 * i, stencil=i % 2) for i in range(8)]
    ex = FakeExecutor()
    sch = SV.Scheduler(ex, budget_bytes=1 << 30, max_active=4, sweeps_per_step=5, tol=1e-8,
                       clock=Clock())
    done = sch.run(_tickets(reqs))
    assert sorted(t.req.rid for t in done) == list(range(8))
    assert all(t.status == SV.DONE and t.rel_residual <= 1e-8 for t in done)
    assert sorted(ex.released) == list(range(8))
    assert sch.used == 0 and sch.stats.completed == 8
    assert all(t.latency_s >= 0 and t.finished_s >= t.admitted_s >= t.req.arrival_s for t in done)
    assert max(len(s) for s in ex.steps) <= 4


def test_budget_limits_what_is_resident():
    reqs = [_req(i, (6, 6, 6)) for i in range(6)]
    per = FakeExecutor().bytes_needed(reqs[0])
    ex = FakeExecutor()
    sch = SV.Scheduler(ex, budget_bytes=2 * per + per // 2, max_active=100, sweeps_per_step=3,
                       clock=Clock())
    sch.run(_tickets(reqs))
    assert max(len(s) for s in ex.steps) == 2          # memory, not slots, limits
    assert sch.stats.peak_bytes <= 2 * per + per // 2
    assert ex.admitted == list(range(6))               # FIFO admission


def test_fifo_head_blocks_smaller_requests():
    big = _req(0, (10, 10, 10))
    small = [_req(i, (3, 3, 3)) for i in (1, 2)]
    per_big = FakeExecutor().bytes_needed(big)
    ex = FakeExecutor()
    sch = SV.Scheduler(ex, budget_bytes=per_big, max_active=8, sweeps_per_step=4, clock=Clock())
    sch.run(_tickets([big] + small))
    assert ex.admitted == [0, 1, 2]
    assert ex.steps[0] == [0]                          # the small ones waited behind the head


def test_failure_states():
    reqs = [_req(0, (4, 4, 4)), _req(1, (5, 4, 4)), _req(2, (40, 40, 40)), _req(3, (4, 4, 5))]
    per = FakeExecutor().bytes_needed(reqs[1])
    tickets = _tickets(reqs, nan_rid=1)
    tickets[3].cancel = True
    ex = FakeExecutor()
    sch = SV.Scheduler(ex, budget_bytes=20 * per, max_active=4, sweeps_per_step=2, tol=1e-8,
                       max_sweeps=4, clock=Clock())
    done = {t.req.rid: t for t in sch.run(tickets)}
    assert done[1].status == SV.DIVERGED and not math.isfinite(done[1].rel_residual)
    assert done[2].status == SV.REJECTED                # larger than the whole budget
    assert done[3].status == SV.CANCELLED
    assert done[0].status == SV.NOT_CONVERGED and done[0].sweeps == 4
    assert sch.used == 0 and sch.stats.failed == 4


def test_latency_statistics():
    reqs = [_req(i, (4, 4, 4), arrival=0.0) for i in range(5)]
    sch = SV.Scheduler(FakeExecutor(), budget_bytes=1 << 30, max_active=2, sweeps_per_step=10,
                       clock=Clock(dt=0.01))
    sch.run(_tickets(reqs))
    s = sch.stats.summary(0.0, max(t.finished_s for t in sch.finished))
    assert s["completed"] == 5 and s["p99_latency_s"] >= s["p50_latency_s"] > 0
    assert np.isclose(s["patches_per_s"], 5 / s["span_s"])
