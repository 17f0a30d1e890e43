"""colsten oracle -- TEST INFRASTRUCTURE ONLY.

Python face of the sequential C oracle in ``colsten_oracle.c`` (built with gcc,
``-O2 -ffp-contract=off``).  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark import this module; the GPU library and its
binding never do, and this module imports nothing from them.

Every array argument is a halo'd numpy array in C order with x contiguous:
shape ``(ny+2, px)`` in 2D and ``(nz+2, ny+2, px)`` in 3D, where the row pitch
``px >= nx+2`` may include padding (a view ``a[..., :nx+2]`` of a wider array
is accepted; the strides are read from the array).  The halo holds the
Dirichlet boundary values.  Function-by-function citations of the paper
(Hazelwood & Weinzierl, arXiv:1810.04033) are in the C source.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "colsten_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")  # the same source with -fopenmp
_lib = None
_openmp = False

FD, Q1 = 0, 1


def build(force=True, openmp=False):
    """Compile the oracle with gcc (no FMA contraction, no fast-math); with
    openmp, the same source with -fopenmp (the colour passes and Jacobi sweeps
    then run one parallel loop per colour, Sec. 3)."""
    out = _LIB_OMP if openmp else _LIB
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(_SRC):
        return out
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    cmd.insert(1, "-fopenmp" if openmp else "-Wno-unknown-pragmas")
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def set_openmp(flag):
    """Route the calls below to the OpenMP build (True) or the sequential one
    (False, the default).  Both give the same results bit for bit."""
    global _lib, _openmp
    if bool(flag) != _openmp:
        _openmp = bool(flag)
        _lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    alt = os.environ.get("COLSTEN_ORACLE_LIB")  # a deliberately mutated build (pin tests)
    if alt:
        lib = ctypes.CDLL(alt)
    else:
        lib = ctypes.CDLL(build(force=False, openmp=_openmp))
    i32, i64, f64, vp = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    geo = [i32, i32, i32, i64, i64, i64, i64, i64, f64]
    lib.og_weight.restype = f64
    lib.og_weight.argtypes = [i32, i32, i32, i32, i32]
    lib.og_num_colours.restype = i32
    lib.og_num_colours.argtypes = [i32, i32]
    lib.og_colour.restype = i32
    lib.og_colour.argtypes = [i32, i32, i32, i64, i64, i64]
    lib.og_colouring_valid.restype = i32
    lib.og_colouring_valid.argtypes = [i32, i32, i32, i64]
    for name in ("og_colour_pass_f64", "og_colour_pass_f32"):
        getattr(lib, name).restype = None
        getattr(lib, name).argtypes = geo + [vp, vp, i32]
    lib.og_update_points_f64.restype = None
    lib.og_update_points_f64.argtypes = geo + [vp, vp, vp, i64]
    for name in ("og_gs_sweeps_f64", "og_gs_sweeps_f32"):
        getattr(lib, name).restype = None
        getattr(lib, name).argtypes = geo + [vp, vp, i32]
    for name in ("og_lex_sweeps_f64", "og_lex_sweeps_f32"):
        getattr(lib, name).restype = None
        getattr(lib, name).argtypes = geo + [vp, vp, i32]
    lib.og_gs_sweeps_cost_f64.restype = None
    lib.og_gs_sweeps_cost_f64.argtypes = geo + [vp, vp, i32, i32, i32, f64, f64, f64]
    for name in ("og_jacobi_sweeps_f64", "og_jacobi_sweeps_f32"):
        getattr(lib, name).restype = None
        getattr(lib, name).argtypes = geo + [vp, vp, vp, f64, i32, i64]
    lib.og_residual_f64.restype = None
    lib.og_residual_f64.argtypes = geo + [vp, vp, vp, vp]
    lib.og_residual_f32in.restype = None
    lib.og_residual_f32in.argtypes = geo + [vp, vp, vp]
    lib.og_q1_kref.restype = f64
    lib.og_q1_kref.argtypes = [i32, i32]
    lib.og_q1_apply_cellwise.restype = None
    lib.og_q1_apply_cellwise.argtypes = [i32, i64, i64, i64, i64, i64, vp, vp]
    lib.og_q1_apply_cellwise_coloured.restype = None
    lib.og_q1_apply_cellwise_coloured.argtypes = [i32, i64, i64, i64, i64, i64, vp, vp]
    lib.og_apply_stencil.restype = None
    lib.og_apply_stencil.argtypes = [i32, i32, i64, i64, i64, i64, i64, vp, vp]
    lib.og_nd_sweeps_f64.restype = None
    lib.og_nd_sweeps_f64.argtypes = geo + [vp, vp, i32, i64]
    lib.og_restrict_f64.restype = None
    lib.og_restrict_f64.argtypes = [i32, i64, i64, i64, i64, i64, i64, i64, vp, vp, vp]
    lib.og_prolong_add_f64.restype = None
    lib.og_prolong_add_f64.argtypes = [i32, i64, i64, i64, i64, i64, i64, i64, vp, vp]
    _lib = lib
    return lib


def _geometry(a, dim):
    """(nx, ny, nz, sy, sz) of a halo'd array (element strides)."""
    if a.ndim != dim:
        raise ValueError("array rank %d does not match dim %d" % (a.ndim, dim))
    it = a.itemsize
    if a.strides[-1] != it:
        raise ValueError("x must be the contiguous axis")
    nx = a.shape[-1] - 2
    ny = a.shape[-2] - 2
    sy = a.strides[-2] // it
    if dim == 3:
        nz = a.shape[-3] - 2
        sz = a.strides[-3] // it
    else:
        nz, sz = 1, 0
    return nx, ny, nz, sy, sz


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _span(a):
    """Number of elements between the first and one past the last element."""
    it = a.itemsize
    return (sum((s - 1) * st for s, st in zip(a.shape, a.strides)) // it) + 1


def _args(u, dim, stencil, parity, h):
    nx, ny, nz, sy, sz = _geometry(u, dim)
    return [dim, stencil, parity, nx, ny, nz, sy, sz, float(h)]


def _check_same(u, *others):
    for o in others:
        if o is None:
            continue
        if o.shape != u.shape or o.strides != u.strides or o.dtype != u.dtype:
            raise ValueError("arrays must share shape, strides and dtype")


def weight(stencil, dim, ox, oy, oz=0):
    return _load().og_weight(stencil, dim, ox, oy, oz)


def num_colours(stencil, dim):
    return _load().og_num_colours(stencil, dim)


def colour(stencil, dim, parity, i, j, k=1):
    return _load().og_colour(stencil, dim, parity, i, j, k)


def colouring_valid(stencil, dim, n, force_red_black=False):
    return bool(_load().og_colouring_valid(stencil, dim, 1 if force_red_black else 0, n))


def colour_pass(u, b, colour_id, *, dim, stencil, h, parity=0):
    """One Gauss-Seidel colour pass, in situ on u (float64 or float32)."""
    _check_same(u, b)
    lib = _load()
    fn = lib.og_colour_pass_f64 if u.dtype == np.float64 else lib.og_colour_pass_f32
    fn(*_args(u, dim, stencil, parity, h), _ptr(u), _ptr(b), int(colour_id))


def update_points(u, b, flat_idx, *, dim, stencil, h, parity=0):
    """Point updates at the given flat element offsets, in the given order."""
    _check_same(u, b)
    idx = np.ascontiguousarray(flat_idx, dtype=np.int64)
    _load().og_update_points_f64(*_args(u, dim, stencil, parity, h), _ptr(u), _ptr(b),
                                 _ptr(idx), int(idx.size))


def gs_sweeps(u, b, nsweeps, *, dim, stencil, h, parity=0):
    """nsweeps Gauss-Seidel sweeps (all colours in canonical order), in situ."""
    _check_same(u, b)
    lib = _load()
    fn = lib.og_gs_sweeps_f64 if u.dtype == np.float64 else lib.og_gs_sweeps_f32
    fn(*_args(u, dim, stencil, parity, h), _ptr(u), _ptr(b), int(nsweeps))


def lex_sweeps(u, b, nsweeps, *, dim, stencil, h):
    """nsweeps lexicographic Gauss-Seidel sweeps (z-y-x order, in place)."""
    _check_same(u, b)
    lib = _load()
    fn = lib.og_lex_sweeps_f64 if u.dtype == np.float64 else lib.og_lex_sweeps_f32
    fn(*_args(u, dim, stencil, 0, h), _ptr(u), _ptr(b), int(nsweeps))


def nd_sweeps(u, b, nsweeps, *, dim, stencil, h, leaf=16):
    """Gauss-Seidel in the nested-dissection ordering of Sec. 3 (the reading of
    og_nd_sweeps_f64: boxes with every edge <= leaf are leaves), float64."""
    _check_same(u, b)
    if u.dtype != np.float64:
        raise ValueError("nested dissection sweeps are float64")
    _load().og_nd_sweeps_f64(*_args(u, dim, stencil, 0, h), _ptr(u), _ptr(b), int(nsweeps), int(leaf))


def gs_sweeps_cost(u, b, nsweeps, kmax, hetero, *, dim, stencil, h, parity=0,
                   z=0.0, a=1.0 / 1024.0, c=1.0 / 128.0):
    """FP64 sweeps with the expensive stencil evaluation S(k), in situ."""
    _check_same(u, b)
    assert u.dtype == np.float64
    lib = _load()
    lib.og_gs_sweeps_cost_f64(*_args(u, dim, stencil, parity, h), _ptr(u), _ptr(b), int(nsweeps),
                              int(kmax), int(hetero), float(z), float(a), float(c))


def _like(u):
    """A zero array with u's shape, dtype and element strides (own buffer)."""
    flat = np.zeros(_span(u), dtype=u.dtype)
    return np.lib.stride_tricks.as_strided(flat, shape=u.shape, strides=u.strides), flat


def jacobi_sweeps(u, b, nsweeps, omega, *, dim, stencil, h):
    """nsweeps weighted Jacobi sweeps; the result is left in u."""
    _check_same(u, b)
    _, flat = _like(u)
    lib = _load()
    fn = lib.og_jacobi_sweeps_f64 if u.dtype == np.float64 else lib.og_jacobi_sweeps_f32
    fn(*_args(u, dim, stencil, 0, h), _ptr(u), _ptr(b), _ptr(flat),
       float(omega), int(nsweeps), int(flat.size))


def residual(u, b, *, dim, stencil, h, want_r=False):
    """r = b - S u / h^2 and (||r||_2, max|r|, ||b||_2) over the interior."""
    _check_same(u, b)
    norms = np.zeros(3, dtype=np.float64)
    lib = _load()
    if u.dtype == np.float32:
        if want_r:
            raise ValueError("r is only returned for float64 grids")
        lib.og_residual_f32in(*_args(u, dim, stencil, 0, h), _ptr(u), _ptr(b), _ptr(norms))
        return norms
    r = _like(u)[0] if want_r else None
    lib.og_residual_f64(*_args(u, dim, stencil, 0, h), _ptr(u), _ptr(b),
                        _ptr(r) if r is not None else None, _ptr(norms))
    return (norms, r) if want_r else norms


def apply_stencil(u, *, dim, stencil):
    """(S u) at interior points (dimensionless stencil, h = 1); halo entries 0."""
    out = _like(u)[0]
    nx, ny, nz, sy, sz = _geometry(u, dim)
    _load().og_apply_stencil(dim, stencil, nx, ny, nz, sy, sz, _ptr(u), _ptr(out))
    return out


def q1_apply_cellwise(u, *, dim):
    """(S u) at interior points by element-wise accumulation; halo entries invalid."""
    out = _like(u)[0]
    nx, ny, nz, sy, sz = _geometry(u, dim)
    _load().og_q1_apply_cellwise(dim, nx, ny, nz, sy, sz, _ptr(u), _ptr(out))
    return out


def q1_apply_cellwise_coloured(u, *, dim):
    """(S u) at interior points by element-wise accumulation in 2^d cell-colour
    passes (each vertex receives its cell contributions in colour order)."""
    out = _like(u)[0]
    nx, ny, nz, sy, sz = _geometry(u, dim)
    _load().og_q1_apply_cellwise_coloured(dim, nx, ny, nz, sy, sz, _ptr(u), _ptr(out))
    return out


def q1_kref(dim, ndiff):
    return _load().og_q1_kref(dim, ndiff)


def interior(a):
    """The interior view of a halo'd array."""
    if a.ndim == 2:
        return a[1:-1, 1:a.shape[1] - 1]
    return a[1:-1, 1:-1, 1:a.shape[2] - 1]


def _pow2_at_least(v):
    """Smallest power of two >= v (1.0 for v <= 0)."""
    if not v > 0.0:
        return 1.0
    p = 1.0
    while p < v:
        p *= 2.0
    while p / 2.0 >= v:
        p /= 2.0
    return p


def ir_solve(b, tol, *, dim, stencil, h, inner_sweeps, max_outer, x0=None):
    """FP32 Gauss-Seidel sweeps inside FP64 iterative refinement.

    Step i: r_i = b - A x_i in FP64; stop when ||r_i||_2 / ||b||_2 <= tol;
    r32 = fl32(r_i / s_i); inner_sweeps FP32 sweeps on A e = r32 from e = 0;
    x_{i+1} = x_i + s_i e in FP64.  The scale s_i is the smallest power of two
    >= max |r_{i-1}|, with r_{-1} = r_0 (so the residual and its FP32 copy can
    be formed in one pass).  Returns (x, history of relative residuals, outer
    steps taken).
    """
    x = np.zeros_like(b) if x0 is None else x0.copy()
    hist = []
    norms = residual(x, b, dim=dim, stencil=stencil, h=h)
    s = _pow2_at_least(norms[1])
    for it in range(max_outer + 1):
        norms, r = residual(x, b, dim=dim, stencil=stencil, h=h, want_r=True)
        rel = norms[0] / norms[2] if norms[2] > 0 else norms[0]
        hist.append(rel)
        if rel <= tol or it == max_outer:
            return x, hist, it
        r32 = (r / s).astype(np.float32)
        e = np.zeros_like(r32)
        gs_sweeps(e, r32, inner_sweeps, dim=dim, stencil=stencil, h=h)
        inner = interior(x)
        inner += s * interior(e).astype(np.float64)
        s = _pow2_at_least(norms[1])
    return x, hist, max_outer


# ---------------------------------------------------------------------------
# Geometric multigrid with the coloured sweep as smoother (the transfers are
# defined in colsten_oracle.c).  FP64 only.
# ---------------------------------------------------------------------------
def _interior_n(a, dim):
    nx, ny, nz, _, _ = _geometry(a, dim)
    return (nx, ny) if dim == 2 else (nx, ny, nz)


def _check_pair(fine, coarse, dim):
    if fine.dtype != np.float64 or coarse.dtype != np.float64:
        raise ValueError("multigrid transfers are float64")
    nf, nc = _interior_n(fine, dim), _interior_n(coarse, dim)
    if any(f != 2 * c + 1 for f, c in zip(nf, nc)):
        raise ValueError("fine n %s is not 2 * coarse n + 1 (coarse %s)" % (nf, nc))


def restrict(r, bc, uc, *, dim):
    """bc <- full weighting of the fine residual r at the coarse interior;
    uc <- 0 at the coarse interior (halos untouched)."""
    _check_pair(r, bc, dim)
    _check_same(bc, uc)
    nxc, nyc, nzc, syc, szc = _geometry(bc, dim)
    _, _, _, syf, szf = _geometry(r, dim)
    _load().og_restrict_f64(dim, nxc, nyc, nzc, syc, szc, syf, szf, _ptr(r), _ptr(bc), _ptr(uc))


def prolong_add(uc, uf, *, dim):
    """uf <- uf + d-linear interpolation of uc (coarse halo included) at the
    fine interior."""
    _check_pair(uf, uc, dim)
    nxf, nyf, nzf, syf, szf = _geometry(uf, dim)
    _, _, _, syc, szc = _geometry(uc, dim)
    _load().og_prolong_add_f64(dim, nxf, nyf, nzf, syf, szf, syc, szc, _ptr(uc), _ptr(uf))


def mg_coarsens(n):
    """Whether a grid of interior sizes n has a coarser level: every axis odd
    and at least 3."""
    return all(v % 2 == 1 and v >= 3 for v in n)


def mg_vcycle(u, b, *, dim, stencil, h, nu1=2, nu2=2, coarse_sweeps=2, parity=0):
    """One V(nu1, nu2)-cycle on A u = b in place: nu1 coloured Gauss-Seidel
    sweeps, residual, restriction, the cycle on the coarse correction equation
    (h doubled, zero initial guess and zero Dirichlet halo), prolongation added
    to u, nu2 sweeps; on a grid that does not coarsen, coarse_sweeps sweeps."""
    n = _interior_n(u, dim)
    if not mg_coarsens(n):
        gs_sweeps(u, b, coarse_sweeps, dim=dim, stencil=stencil, h=h, parity=parity)
        return
    gs_sweeps(u, b, nu1, dim=dim, stencil=stencil, h=h, parity=parity)
    _, r = residual(u, b, dim=dim, stencil=stencil, h=h, want_r=True)
    shape = tuple((v - 1) // 2 + 2 for v in reversed(n))
    uc = np.zeros(shape, dtype=np.float64)
    bc = np.zeros(shape, dtype=np.float64)
    restrict(r, bc, uc, dim=dim)
    mg_vcycle(uc, bc, dim=dim, stencil=stencil, h=2.0 * h, nu1=nu1, nu2=nu2,
              coarse_sweeps=coarse_sweeps, parity=parity)
    prolong_add(uc, u, dim=dim)
    gs_sweeps(u, b, nu2, dim=dim, stencil=stencil, h=h, parity=parity)
