"""The request server on the GPU: a mixed stream of patch solves (both
stencils, FP64 and FP32-in-FP64 refinement) converges, every result passes the
oracle's FP64 residual check, and a request's result is the same alone and in
the mix."""
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_1810_04033_amd import inputs as I
from paper_1810_04033_amd import serve as SV

pytestmark = pytest.mark.gpu


def _serve(reqs, k=10, budget=1 << 30, max_active=64):
    tickets = SV.make_tickets(reqs)
    t0 = time.perf_counter()
    sch = SV.Scheduler(SV.GpuExecutor(keep_results=True), budget_bytes=budget,
                       max_active=max_active, sweeps_per_step=k, tol=1e-8,
                       clock=lambda: time.perf_counter() - t0)
    return {t.req.rid: t for t in sch.run(tickets)}, sch


def test_mixed_stream_converges_and_is_mix_independent():
    reqs = I.request_stream(11, 24, 2000.0, edge_lo=8, edge_hi=24)
    assert {r.stencil for r in reqs} == {0, 1} and {r.mixed for r in reqs} == {False, True}
    done, sch = _serve(reqs, budget=40 << 20, max_active=12)
    assert all(t.status == SV.DONE for t in done.values())
    assert sch.stats.max_active > 1
    for r in reqs:
        t = done[r.rid]
        nx, ny, nz = r.n
        b = I.halo_array(I.uniform_field(r.rhs_seed, (nz, ny, nx)))
        nr = O.residual(t.result, b, dim=3, stencil=r.stencil, h=1.0 / (max(r.n) + 1))
        assert nr[0] / nr[2] <= 1e-8
    for r in (reqs[0], reqs[5], reqs[13]):
        alone, _ = _serve([I.Request(r.rid, 0.0, r.n, r.stencil, r.mixed, r.rhs_seed)])
        a = alone[r.rid]
        assert a.sweeps == done[r.rid].sweeps
        assert np.array_equal(a.result, done[r.rid].result)


def test_workload_sizes_stream_is_mix_independent():
    """32 requests drawn as the serving workload draws them (edges log-uniform
    in [16, 128], aspect <= 4, both stencils, FP64 and refinement): every one
    converges under the oracle's FP64 residual, and for each of the four
    (stencil, precision) classes the request with the widest x extent -- all in
    the large tile class, several with an edge above 64 -- gives the same
    sweeps and the same iterate, bit for bit, alone and in the mix."""
    reqs = I.request_stream(21, 32, 2000.0)
    probes = []
    for cls in ((0, False), (0, True), (1, False), (1, True)):
        members = [r for r in reqs if (r.stencil, r.mixed) == cls]
        assert members
        probes.append(max(members, key=lambda r: r.n[0]))
    assert all(p.n[0] > 40 for p in probes)
    assert sum(max(p.n) > 64 for p in probes) >= 3
    done, sch = _serve(reqs, k=20, budget=4 << 30, max_active=64)
    assert all(t.status == SV.DONE for t in done.values())
    assert sch.stats.max_active > 8
    for r in reqs:
        t = done[r.rid]
        nx, ny, nz = r.n
        b = I.halo_array(I.uniform_field(r.rhs_seed, (nz, ny, nx)))
        nr = O.residual(t.result, b, dim=3, stencil=r.stencil, h=1.0 / (max(r.n) + 1))
        assert nr[0] / nr[2] <= 1e-8
    for r in probes:
        alone, _ = _serve([I.Request(r.rid, 0.0, r.n, r.stencil, r.mixed, r.rhs_seed)], k=20)
        a = alone[r.rid]
        assert a.sweeps == done[r.rid].sweeps
        assert np.array_equal(a.result, done[r.rid].result)
