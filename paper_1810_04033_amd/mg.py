"""Geometric multigrid V-cycles whose smoother is the coloured Gauss-Seidel
sweep (the paper names multigrid as the setting its smoothers serve, Sec. 1).

A cycle on a level is: nu1 sweeps, the residual r = b - A u, full weighting
of r into the right-hand side of the next coarser level (whose iterate is set
to zero), the cycle there, d-linear interpolation of the coarse correction
added to u, nu2 sweeps.  A level coarsens while every interior size is odd and
at least 3 (n = 2 n_c + 1, h_c = 2 h); the coarsest level gets coarse_sweeps
sweeps.  Sizes 2^m - 1 therefore coarsen down to one point.  The host only
enqueues library calls on one stream; every step runs in the library's
kernels (sweeps, residual, cs_restrict, cs_prolong_add), and the only host
synchronisation is the read-back of the residual norms in solve().
"""
import math

from . import colsten as C
from .solve import SolveResult


def coarsens(n):
    """Whether interior sizes n have a coarser level."""
    return all(v % 2 == 1 and v >= 3 for v in n)


class _Level:
    def __init__(self, grid, tmp, r):
        self.grid, self.tmp, self.r = grid, tmp, r


class Multigrid:
    """The level hierarchy below a fine grid; the fine grid's u and b are the
    caller's, the coarser levels' arrays are allocated here (zero halos: the
    coarse equations are for corrections with homogeneous boundary values)."""

    def __init__(self, grid, *, nu1=2, nu2=2, coarse_sweeps=2):
        if min(nu1, nu2, coarse_sweeps) < 0:
            raise ValueError("sweep counts must be >= 0")
        self.nu1, self.nu2, self.coarse_sweeps = int(nu1), int(nu2), int(coarse_sweeps)
        dim = grid.dim
        n = tuple(int(grid.desc.n[a]) for a in range(dim))
        u = grid.u
        self.levels = [_Level(grid, C.grid_like(u), C.grid_like(u) if coarsens(n) else None)]
        h = grid.h
        while coarsens(n):
            n = tuple((v - 1) // 2 for v in n)
            h = 2.0 * h
            uc = C.empty_grid(n, dtype=u.dtype, device=u.device)
            bc = C.empty_grid(n, dtype=u.dtype, device=u.device)
            gc = C.Grid(uc, bc, dim=dim, stencil=grid.stencil, h=h, parity=grid.parity)
            self.levels.append(_Level(gc, C.grid_like(uc), C.grid_like(uc) if coarsens(n) else None))

    @property
    def depth(self):
        return len(self.levels)

    def cycle(self, stream=None):
        """Enqueue one V(nu1, nu2)-cycle on the fine grid."""
        lv = self.levels
        for a, b in zip(lv[:-1], lv[1:]):
            a.grid.gs(self.nu1, tmp=a.tmp, stream=stream)
            a.grid.residual(r=a.r, stream=stream, want_norms=False)
            C.restrict(a.grid, a.r, b.grid, stream)
        lv[-1].grid.gs(self.coarse_sweeps, tmp=lv[-1].tmp, stream=stream)
        for a, b in zip(reversed(lv[:-1]), reversed(lv[1:])):
            C.prolong_add(b.grid, a.grid, stream)
            a.grid.gs(self.nu2, tmp=a.tmp, stream=stream)

    def capture(self):
        """Record one V-cycle into a HIP graph (one replay call per cycle
        instead of a library call per kernel); cycle_graph() replays it."""
        if getattr(self, "graph", None) is None:
            self.graph = C.Graph.record(lambda s: self.cycle(stream=s), keep=(self.levels,))
        return self.graph

    def cycle_graph(self, stream=None):
        """Enqueue one V-cycle as a replay of the captured graph."""
        self.capture().launch(stream)

    def solve(self, tol, *, max_cycles=200, stream=None, progress=None, graph=False):
        """V-cycles until ||b - A u||_2 / ||b||_2 <= tol.  Returns a
        SolveResult whose `outer` counts the cycles and `sweeps` the fine-grid
        sweeps; progress(cycles, rel) is called after every cycle.  graph:
        replay a captured cycle instead of enqueueing its calls."""
        fine = self.levels[0].grid

        def rel_of(t):
            v = t.cpu().tolist()
            return v[0] / v[2] if v[2] > 0 else v[0]

        rel = rel_of(fine.residual(stream=stream))
        hist = [rel]
        cycles = 0
        while rel > tol and cycles < max_cycles:
            if graph:
                self.cycle_graph(stream)
            else:
                self.cycle(stream)
            cycles += 1
            rel = rel_of(fine.residual(stream=stream))
            hist.append(rel)
            if progress is not None:
                progress(cycles, rel)
            if not math.isfinite(rel):
                break
        per = self.nu1 + self.nu2 if self.depth > 1 else self.coarse_sweeps
        return SolveResult(rel <= tol, cycles * per, cycles, rel, hist)

    def close(self):
        if getattr(self, "graph", None) is not None:
            self.graph.close()
            self.graph = None
        for lv in self.levels[1:]:
            lv.grid.close()
