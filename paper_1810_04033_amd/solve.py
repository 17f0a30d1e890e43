"""Solves built from the C-ABI calls: Gauss-Seidel to a tolerance in FP64, and
FP32 sweeps inside FP64 iterative refinement.

Both loops run on the host and enqueue library calls on one stream; the only
host synchronisation is the read-back of the three residual norms at each
convergence check.  All arithmetic happens in the library's kernels.
"""
import math
from dataclasses import dataclass, field

import torch

from . import colsten as C


def pow2_at_least(v):
    """Smallest power of two >= v (1.0 for v <= 0 or non-finite v)."""
    if not (v > 0.0) or not math.isfinite(v):
        return 1.0
    m, e = math.frexp(v)  # v = m * 2**e, 0.5 <= m < 1
    return math.ldexp(1.0, e - 1) if m == 0.5 else math.ldexp(1.0, e)


@dataclass
class SolveResult:
    converged: bool
    sweeps: int                 # Gauss-Seidel sweeps (inner sweeps for refinement)
    outer: int = 0              # refinement steps
    rel_residual: float = float("nan")
    history: list = field(default_factory=list)


def gs_solve(grid, tol, *, check_every=10, tmp=None, max_sweeps=10 ** 7, stream=None,
             progress=None):
    """FP64 (or FP32) Gauss-Seidel sweeps until ||b - A u|| / ||b|| <= tol,
    checked every `check_every` sweeps.  progress(sweeps, rel) is called
    after every check when given."""
    norms = grid.residual(stream=stream)
    n = norms.cpu().tolist()
    rel = n[0] / n[2] if n[2] > 0 else n[0]
    hist = [rel]
    sweeps = 0
    while rel > tol and sweeps < max_sweeps:
        step = min(check_every, max_sweeps - sweeps)
        grid.gs(step, tmp=tmp, stream=stream)
        sweeps += step
        n = grid.residual(stream=stream).cpu().tolist()
        rel = n[0] / n[2] if n[2] > 0 else n[0]
        hist.append(rel)
        if progress is not None:
            progress(sweeps, rel)
        if not math.isfinite(rel):
            break
    return SolveResult(rel <= tol, sweeps, 0, rel, hist)


def ir_solve(g64, g32, tol, *, inner_sweeps, tmp32=None, max_outer=10 ** 6, stream=None,
             progress=None, inner=None):
    """FP32 Gauss-Seidel sweeps inside FP64 iterative refinement.

    Step i: r_i = b - A x_i (FP64) with r32 = fl32(r_i / s_i) and e = 0 in the
    same pass; stop when ||r_i|| / ||b|| <= tol; `inner_sweeps` FP32 sweeps on
    A e = r32; x_{i+1} = x_i + s_i e (FP64).  s_i is the smallest power of two
    >= max |r_{i-1}| (r_{-1} = r_0, from one plain residual first).
    inner: None, or a callable inner(stream) that replaces the inner sweeps
    by another FP32 solve of A e = r32 on g32 from e = 0 (e.g. multigrid
    cycles); `sweeps` then adds inner_sweeps per call."""
    norms = torch.zeros(3, dtype=torch.float64, device=g64.u.device)
    C.cs_residual(g64.handle, 0, norms.data_ptr(), stream)
    n = norms.cpu().tolist()
    scale = pow2_at_least(n[1])
    hist = []
    sweeps = 0
    for outer in range(max_outer + 1):
        C.cs_ir_residual(g64.handle, g32.handle, scale, norms.data_ptr(), stream)
        n = norms.cpu().tolist()
        rel = n[0] / n[2] if n[2] > 0 else n[0]
        hist.append(rel)
        if progress is not None:
            progress(sweeps, rel)
        if rel <= tol or not math.isfinite(rel) or outer == max_outer:
            return SolveResult(rel <= tol, sweeps, outer, rel, hist)
        if inner is None:
            g32.gs(inner_sweeps, tmp=tmp32, stream=stream)
        else:
            inner(stream)
        sweeps += inner_sweeps
        C.cs_ir_update(g64.handle, g32.handle, scale, stream)
        scale = pow2_at_least(n[1])
    return SolveResult(False, sweeps, max_outer, hist[-1] if hist else float("nan"), hist)
