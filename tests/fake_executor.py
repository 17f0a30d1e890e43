"""A CPU stand-in executor for the scheduler tests (test-only; the library
never imports it).  It advances each admitted patch with the oracle."""
import numpy as np

from oracle import oracle as O
from paper_1810_04033_amd import inputs as I


class FakeExecutor:
    def __init__(self, bytes_per_point=24):
        self.bpp = bytes_per_point
        self.admitted = []
        self.released = []
        self.steps = []

    def bytes_needed(self, req):
        nx, ny, nz = req.n
        return (nx + 2) * (ny + 2) * (nz + 2) * self.bpp

    def admit(self, t):
        nx, ny, nz = t.req.n
        h = 1.0 / (max(t.req.n) + 1)
        t.state = {"u": I.halo_array(np.zeros((nz, ny, nx))), "b": I.halo_array(t.rhs), "h": h}
        self.admitted.append(t.req.rid)

    def release(self, t):
        self.released.append(t.req.rid)

    def step(self, tickets, k):
        self.steps.append([t.req.rid for t in tickets])
        rels = []
        for t in tickets:
            st = t.state
            O.gs_sweeps(st["u"], st["b"], k, dim=3, stencil=t.req.stencil, h=st["h"])
            t.sweeps += k
            nr = O.residual(st["u"], st["b"], dim=3, stencil=t.req.stencil, h=st["h"])
            rels.append(nr[0] / nr[2] if nr[2] > 0 else nr[0])
        return rels
