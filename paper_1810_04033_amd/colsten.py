"""Python binding of libcolsten (ctypes; argument marshalling only).

The functions carry the C names of include/colsten.h and raise ColstenError on
a non-zero status.  Every step of the computation runs in the HIP kernels of
libcolsten.so; there is no CPU fallback: if the library is missing, loading it
raises.  torch is imported first so that the library binds to the HIP runtime
torch already loaded (one runtime per process: torch's tensors and streams
are valid in the library).

``Grid`` wraps a handle around caller-owned torch tensors; ``empty_grid``
allocates halo'd arrays whose interior rows start on a 128-byte boundary.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcolsten.so")

CS_OK, CS_EINVAL, CS_ENOMEM, CS_EHIP, CS_EUNSUPPORTED = 0, 1, 2, 3, 4
CS_F64, CS_F32 = 0, 1
CS_FD, CS_Q1 = 0, 1
CS_PASS_AUTO, CS_PASS_ONE, CS_PASS_TWO = 0, 1, 2

_STATUS = {0: "CS_OK", 1: "CS_EINVAL", 2: "CS_ENOMEM", 3: "CS_EHIP", 4: "CS_EUNSUPPORTED"}


class ColstenError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


class cs_grid_desc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("stencil", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("parity", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("stride", ctypes.c_int64 * 3),
        ("h", ctypes.c_double),
    ]


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "cs_grid_create": (ctypes.c_int, [ctypes.POINTER(cs_grid_desc), ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_void_p)]),
    "cs_grid_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "cs_num_colours": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "cs_gs_fused": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "cs_grid_set_pass_mode": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "cs_gs_sweeps_sync": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "cs_gs_sync_failures": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]),
    "cs_sweeps_per_pass": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "cs_colour_pass": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "cs_gs_sweeps": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "cs_jacobi_sweeps": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "cs_residual": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cs_residual_noalloc": (ctypes.c_int, [ctypes.POINTER(cs_grid_desc), ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cs_fill_uniform": (ctypes.c_int, [ctypes.POINTER(cs_grid_desc), ctypes.c_void_p, ctypes.c_uint64,
                                       ctypes.c_void_p]),
    "cs_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "cs_gs_sweeps_lex": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "cs_gs_sweeps_cost": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_void_p]),
    "cs_ir_residual": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                                      ctypes.c_void_p]),
    "cs_ir_update": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]),
    "cs_gs_sweeps_dep": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "cs_gs_sweeps_nd": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]),
    "cs_restrict": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cs_prolong_add": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cs_batch_create": (ctypes.c_int, [ctypes.POINTER(cs_grid_desc), ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "cs_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "cs_batch_reserve": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_void_p)]),
    "cs_batch_assign": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(cs_grid_desc), ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_void_p]),
    "cs_batch_ir_attach": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(cs_grid_desc),
                                          ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                          ctypes.c_void_p]),
    "cs_batch_ir_residual": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cs_batch_ir_update": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cs_batch_gs_sweeps": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "cs_batch_residual": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "cs_batch_sweeps_per_pass": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "cs_batch_tile_policy": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "cs_batch_colour_policy": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64]),
    "cs_grid_schedule_policy": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                               ctypes.c_int64]),
    "cs_batch_pass_policy": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "cs_batch_resident_policy": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "cs_graph_gs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_void_p)]),
    "cs_graph_batch_gs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "cs_graph_begin": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p)]),
    "cs_graph_end": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "cs_graph_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "cs_graph_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "cs_last_error": (ctypes.c_char_p, []),
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcolsten.so is not built (%s); run `python -m "
                          "paper_1810_04033_amd.build`" % LIB_PATH)
    handle = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(handle, name)
        fn.restype = res
        fn.argtypes = args
    _lib = handle
    return handle


def exported_symbols():
    return sorted(_SIGS)


def _check(status):
    if status != CS_OK:
        raise ColstenError(status, lib().cs_last_error().decode())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def cs_last_error():
    return lib().cs_last_error().decode()


def cs_grid_create(desc, u_ptr, b_ptr):
    out = ctypes.c_void_p()
    _check(lib().cs_grid_create(ctypes.byref(desc), ctypes.c_void_p(u_ptr), ctypes.c_void_p(b_ptr),
                                ctypes.byref(out)))
    return out.value


def cs_grid_destroy(handle):
    _check(lib().cs_grid_destroy(ctypes.c_void_p(handle)))


def cs_num_colours(handle):
    out = ctypes.c_int32()
    _check(lib().cs_num_colours(ctypes.c_void_p(handle), ctypes.byref(out)))
    return out.value


def cs_gs_fused(handle):
    out = ctypes.c_int32()
    _check(lib().cs_gs_fused(ctypes.c_void_p(handle), ctypes.byref(out)))
    return bool(out.value)


def cs_gs_sweeps_sync(handle, nsweeps, stream=None):
    _check(lib().cs_gs_sweeps_sync(ctypes.c_void_p(handle), ctypes.c_int32(nsweeps), _stream(stream)))


def cs_gs_sweeps_dep(handle, nsweeps, stream=None):
    _check(lib().cs_gs_sweeps_dep(ctypes.c_void_p(handle), ctypes.c_int32(nsweeps), _stream(stream)))


def cs_gs_sweeps_nd(handle, nsweeps, leaf, stream=None):
    _check(lib().cs_gs_sweeps_nd(ctypes.c_void_p(handle), ctypes.c_int32(nsweeps), ctypes.c_int32(leaf),
                                 _stream(stream)))


def cs_gs_sync_failures(handle, stream=None):
    out = ctypes.c_int32()
    _check(lib().cs_gs_sync_failures(ctypes.c_void_p(handle), ctypes.byref(out), _stream(stream)))
    return out.value


def cs_grid_set_pass_mode(handle, mode):
    _check(lib().cs_grid_set_pass_mode(ctypes.c_void_p(handle), ctypes.c_int32(mode)))


def cs_sweeps_per_pass(handle, jacobi):
    out = ctypes.c_int32()
    _check(lib().cs_sweeps_per_pass(ctypes.c_void_p(handle), ctypes.c_int32(1 if jacobi else 0),
                                    ctypes.byref(out)))
    return out.value


def cs_colour_pass(handle, colour, stream=None):
    _check(lib().cs_colour_pass(ctypes.c_void_p(handle), int(colour), _stream(stream)))


def cs_gs_sweeps(handle, nsweeps, u_tmp_ptr=0, stream=None):
    _check(lib().cs_gs_sweeps(ctypes.c_void_p(handle), int(nsweeps), ctypes.c_void_p(u_tmp_ptr),
                              _stream(stream)))


def fill_uniform(t, seed, *, dim, stream=None):
    """Fill the interior of the halo'd device tensor t with the seeded
    uniform[-1, 1) field (on the GPU; same values as inputs.uniform_field)."""
    d = describe(t, dim=dim, stencil=CS_FD, h=1.0)
    _check(lib().cs_fill_uniform(ctypes.byref(d), ctypes.c_void_p(t.data_ptr()), ctypes.c_uint64(int(seed)),
                                 _stream(stream)))


def cs_apply(handle, y_ptr, cellwise=0, stream=None):
    _check(lib().cs_apply(ctypes.c_void_p(handle), ctypes.c_void_p(y_ptr), int(cellwise), _stream(stream)))


def cs_gs_sweeps_lex(handle, nsweeps, stream=None):
    _check(lib().cs_gs_sweeps_lex(ctypes.c_void_p(handle), int(nsweeps), _stream(stream)))


def cs_gs_sweeps_cost(handle, nsweeps, kmax, hetero=0, stream=None):
    _check(lib().cs_gs_sweeps_cost(ctypes.c_void_p(handle), int(nsweeps), int(kmax), int(hetero),
                                   _stream(stream)))


def cs_jacobi_sweeps(handle, omega, nsweeps, u_tmp_ptr, stream=None):
    _check(lib().cs_jacobi_sweeps(ctypes.c_void_p(handle), float(omega), int(nsweeps),
                                  ctypes.c_void_p(u_tmp_ptr), _stream(stream)))


def cs_residual(handle, r_ptr, norms_ptr, stream=None):
    _check(lib().cs_residual(ctypes.c_void_p(handle), ctypes.c_void_p(r_ptr), ctypes.c_void_p(norms_ptr),
                             _stream(stream)))


def cs_residual_noalloc(desc, u_ptr, b_ptr, r_ptr, norms_ptr, stream=None):
    _check(lib().cs_residual_noalloc(ctypes.byref(desc), ctypes.c_void_p(u_ptr), ctypes.c_void_p(b_ptr),
                                     ctypes.c_void_p(r_ptr), ctypes.c_void_p(norms_ptr), _stream(stream)))


def cs_ir_residual(h64, h32, scale, norms_ptr, stream=None):
    _check(lib().cs_ir_residual(ctypes.c_void_p(h64), ctypes.c_void_p(h32), float(scale),
                                ctypes.c_void_p(norms_ptr), _stream(stream)))


def cs_ir_update(h64, h32, scale, stream=None):
    _check(lib().cs_ir_update(ctypes.c_void_p(h64), ctypes.c_void_p(h32), float(scale), _stream(stream)))


def cs_restrict(h_fine, r_ptr, h_coarse, stream=None):
    _check(lib().cs_restrict(ctypes.c_void_p(h_fine), ctypes.c_void_p(r_ptr), ctypes.c_void_p(h_coarse),
                             _stream(stream)))


def cs_prolong_add(h_coarse, h_fine, stream=None):
    _check(lib().cs_prolong_add(ctypes.c_void_p(h_coarse), ctypes.c_void_p(h_fine), _stream(stream)))


def restrict(fine, r, coarse, stream=None):
    """coarse.b <- full weighting of r (fine layout) and coarse.u <- 0, at the
    coarse interior."""
    cs_restrict(fine.handle, r.data_ptr(), coarse.handle, stream)


def prolong_add(coarse, fine, stream=None):
    """fine.u <- fine.u + d-linear interpolation of coarse.u (halo included)."""
    cs_prolong_add(coarse.handle, fine.handle, stream)


def cs_batch_create(descs, u_ptrs, b_ptrs, tmp_ptrs):
    n = len(descs)
    arr = (cs_grid_desc * n)(*descs)
    vp = ctypes.c_void_p * n
    out = ctypes.c_void_p()
    _check(lib().cs_batch_create(arr, vp(*u_ptrs), vp(*b_ptrs), vp(*tmp_ptrs), n, ctypes.byref(out)))
    return out.value


def cs_batch_destroy(handle):
    _check(lib().cs_batch_destroy(ctypes.c_void_p(handle)))


def cs_batch_reserve(capacity, partials):
    out = ctypes.c_void_p()
    _check(lib().cs_batch_reserve(int(capacity), int(partials), ctypes.byref(out)))
    return out.value


def cs_batch_assign(handle, descs, u_ptrs, b_ptrs, tmp_ptrs, rows=None, stream=None):
    n = len(descs)
    arr = (cs_grid_desc * max(n, 1))(*descs)
    vp = ctypes.c_void_p * max(n, 1)
    r = None if rows is None else (ctypes.c_int32 * max(n, 1))(*[int(x) for x in rows])
    _check(lib().cs_batch_assign(ctypes.c_void_p(handle), arr, vp(*u_ptrs), vp(*b_ptrs), vp(*tmp_ptrs),
                                 r, n, _stream(stream)))


def cs_batch_ir_attach(handle, descs64, x_ptrs, b_ptrs, stream=None):
    n = len(descs64)
    arr = (cs_grid_desc * max(n, 1))(*descs64)
    vp = ctypes.c_void_p * max(n, 1)
    _check(lib().cs_batch_ir_attach(ctypes.c_void_p(handle), arr, vp(*x_ptrs), vp(*b_ptrs), _stream(stream)))


def cs_batch_ir_residual(handle, scales_ptr, norms_ptr, stream=None):
    _check(lib().cs_batch_ir_residual(ctypes.c_void_p(handle), ctypes.c_void_p(scales_ptr),
                                      ctypes.c_void_p(norms_ptr), _stream(stream)))


def cs_batch_ir_update(handle, scales_ptr, stream=None):
    _check(lib().cs_batch_ir_update(ctypes.c_void_p(handle), ctypes.c_void_p(scales_ptr), _stream(stream)))


def residual_items(n):
    """Residual partial sums a patch of interior shape n = (nx, ny, nz) needs in
    a batch (one per 16 rows)."""
    return (n[1] * n[2] + 15) // 16


def cs_batch_gs_sweeps(handle, nsweeps, stream=None):
    _check(lib().cs_batch_gs_sweeps(ctypes.c_void_p(handle), int(nsweeps), _stream(stream)))


def cs_batch_residual(handle, norms_ptr, stream=None):
    _check(lib().cs_batch_residual(ctypes.c_void_p(handle), ctypes.c_void_p(norms_ptr), _stream(stream)))


def cs_batch_sweeps_per_pass(handle, index):
    out = ctypes.c_int32()
    _check(lib().cs_batch_sweeps_per_pass(ctypes.c_void_p(handle), ctypes.c_int32(index), ctypes.byref(out)))
    return out.value


def cs_batch_pass_policy(stencil, dtype, pair_large):
    _check(lib().cs_batch_pass_policy(ctypes.c_int32(stencil), ctypes.c_int32(dtype),
                                      ctypes.c_int32(int(pair_large))))


def cs_batch_resident_policy(stencil, dtype, enable):
    _check(lib().cs_batch_resident_policy(ctypes.c_int32(stencil), ctypes.c_int32(dtype),
                                          ctypes.c_int32(int(enable))))


def cs_grid_schedule_policy(stencil, dtype, block_max, colour_max, two_min):
    _check(lib().cs_grid_schedule_policy(int(stencil), int(dtype), int(block_max), int(colour_max),
                                         int(two_min)))


def cs_batch_colour_policy(stencil, dtype, max_points):
    _check(lib().cs_batch_colour_policy(int(stencil), int(dtype), int(max_points)))


def cs_batch_tile_policy(stencil, dtype, small_max, mid_max):
    _check(lib().cs_batch_tile_policy(int(stencil), int(dtype), int(small_max), int(mid_max)))


# --------------------------------------------------------------------------
# Tensor helpers
# --------------------------------------------------------------------------

_DT = {torch.float64: CS_F64, torch.float32: CS_F32}


def empty_grid(n, dtype=torch.float64, device="cuda", align_bytes=128):
    """A zeroed halo'd tensor for interior size n = (nx, ny[, nz]).

    The returned view has shape (nz+2, ny+2, nx+2) (or (ny+2, nx+2)); its row
    pitch is a multiple of align_bytes and element x = 1 of every row starts
    on an align_bytes boundary (the base allocation is 256-byte aligned)."""
    n = tuple(int(v) for v in n)
    esz = torch.empty((), dtype=dtype).element_size()
    a = max(1, align_bytes // esz)
    nx = n[0]
    px = ((nx + 2 + a - 1) // a) * a
    shape = tuple(v + 2 for v in reversed(n[1:])) + (nx + 2,)
    rows = 1
    for v in shape[:-1]:
        rows *= v
    off = a - 1
    flat = torch.zeros(off + rows * px, dtype=dtype, device=device)
    strides = []
    acc = px
    for v in reversed(shape[:-1]):
        strides.insert(0, acc)
        acc *= v
    view = flat.as_strided(shape, tuple(strides) + (1,), storage_offset=off)
    return view


def grid_like(t):
    """A zeroed tensor with t's shape, strides and dtype (own storage)."""
    span = 1 + sum((s - 1) * st for s, st in zip(t.shape, t.stride()))
    off = t.storage_offset()
    flat = torch.zeros(off + span, dtype=t.dtype, device=t.device)
    return flat.as_strided(t.shape, t.stride(), storage_offset=off)


def describe(u, *, dim, stencil, h, parity=0):
    """cs_grid_desc of a halo'd tensor (shape and strides read from u)."""
    if u.dim() != dim:
        raise ValueError("tensor rank %d does not match dim %d" % (u.dim(), dim))
    if u.stride(-1) != 1:
        raise ValueError("x must be contiguous")
    d = cs_grid_desc()
    d.dim = dim
    d.stencil = int(stencil)
    d.dtype = _DT[u.dtype]
    d.parity = int(parity)
    d.n[0] = u.shape[-1] - 2
    d.n[1] = u.shape[-2] - 2
    d.n[2] = u.shape[-3] - 2 if dim == 3 else 1
    d.stride[0] = 1
    d.stride[1] = u.stride(-2)
    d.stride[2] = u.stride(-3) if dim == 3 else 0
    d.h = float(h)
    return d


class Grid:
    """A colsten grid bound to caller-owned tensors u (updated) and b."""

    def __init__(self, u, b, *, dim, stencil, h, parity=0):
        if u.shape != b.shape or u.stride() != b.stride() or u.dtype != b.dtype:
            raise ValueError("u and b must share shape, strides and dtype")
        self.u, self.b = u, b
        self.dim, self.stencil, self.h, self.parity = dim, stencil, h, parity
        self.desc = describe(u, dim=dim, stencil=stencil, h=h, parity=parity)
        self.handle = cs_grid_create(self.desc, u.data_ptr(), b.data_ptr())
        self.norms = torch.zeros(3, dtype=torch.float64, device=u.device)

    def close(self):
        if self.handle:
            cs_grid_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_colours(self):
        return cs_num_colours(self.handle)

    @property
    def fused(self):
        return cs_gs_fused(self.handle)

    def gs_sync(self, nsweeps, stream=None):
        """Sweeps in one persistent launch with a device-wide barrier per colour."""
        cs_gs_sweeps_sync(self.handle, nsweeps, stream)

    def gs_dep(self, nsweeps, stream=None):
        """Sweeps in one persistent launch, each tile waiting only for its
        neighbour tiles' previous colour (no barrier between colours)."""
        cs_gs_sweeps_dep(self.handle, nsweeps, stream)

    def gs_nd(self, nsweeps, leaf=16, stream=None):
        """Gauss-Seidel sweeps in the nested-dissection ordering (leaves of
        edge <= leaf), a different iterate from the colouring."""
        cs_gs_sweeps_nd(self.handle, nsweeps, leaf, stream)

    def sync_failures(self, stream=None):
        return cs_gs_sync_failures(self.handle, stream)

    def set_pass_mode(self, mode):
        """CS_PASS_AUTO, CS_PASS_ONE or CS_PASS_TWO: sweeps per pass over memory."""
        cs_grid_set_pass_mode(self.handle, mode)

    def sweeps_per_pass(self, jacobi=False):
        return cs_sweeps_per_pass(self.handle, jacobi)

    def colour_pass(self, colour, stream=None):
        cs_colour_pass(self.handle, colour, stream)

    def gs(self, nsweeps, tmp=None, stream=None):
        cs_gs_sweeps(self.handle, nsweeps, 0 if tmp is None else tmp.data_ptr(), stream)

    def apply(self, y, cellwise=False, stream=None):
        """y = A u at the interior (stencil form, or element-wise by cell colours)."""
        cs_apply(self.handle, y.data_ptr(), 1 if cellwise else 0, stream)

    def gs_lex(self, nsweeps, stream=None):
        """Lexicographic Gauss-Seidel sweeps (hyperplane wavefronts)."""
        cs_gs_sweeps_lex(self.handle, nsweeps, stream)

    def gs_cost(self, nsweeps, kmax, hetero=False, stream=None):
        """Sweeps with the expensive stencil evaluation S(k) (one launch per colour)."""
        cs_gs_sweeps_cost(self.handle, nsweeps, kmax, 1 if hetero else 0, stream)

    def jacobi(self, omega, nsweeps, tmp, stream=None):
        cs_jacobi_sweeps(self.handle, omega, nsweeps, tmp.data_ptr(), stream)

    def residual(self, r=None, norms=None, stream=None, want_norms=True):
        """Enqueue the residual; returns the device tensor of the 3 norms
        (None with want_norms=False, which only fills r)."""
        if not want_norms:
            if r is None:
                raise ValueError("want_norms=False needs r")
            cs_residual(self.handle, r.data_ptr(), 0, stream)
            return None
        out = self.norms if norms is None else norms
        cs_residual(self.handle, 0 if r is None else r.data_ptr(), out.data_ptr(), stream)
        return out


class Graph:
    """A captured sequence of sweeps (HIP graph); launch() replays it."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep  # the captured arrays stay referenced while the graph lives

    @classmethod
    def of_grid(cls, grid, nsweeps, tmp=None, lexicographic=False):
        h = ctypes.c_void_p()
        _check(lib().cs_graph_gs(ctypes.c_void_p(grid.handle), int(nsweeps),
                                 ctypes.c_void_p(0 if tmp is None else tmp.data_ptr()),
                                 1 if lexicographic else 0, ctypes.byref(h)))
        return cls(h.value, (grid, tmp))

    @classmethod
    def of_batch(cls, batch, nsweeps):
        h = ctypes.c_void_p()
        _check(lib().cs_graph_batch_gs(ctypes.c_void_p(batch.handle), int(nsweeps), ctypes.byref(h)))
        return cls(h.value, (batch,))

    @classmethod
    def record(cls, enqueue, keep=()):
        """Capture the library calls enqueue(stream) makes on the capture
        stream it is given (a raw stream handle); keep: objects whose arrays
        the graph uses."""
        s = ctypes.c_void_p()
        _check(lib().cs_graph_begin(ctypes.byref(s)))
        h = ctypes.c_void_p()
        try:
            enqueue(s.value)
        except BaseException:
            if lib().cs_graph_end(s, ctypes.byref(h)) == CS_OK and h.value:
                lib().cs_graph_destroy(h)
            raise
        _check(lib().cs_graph_end(s, ctypes.byref(h)))
        return cls(h.value, keep)

    def launch(self, stream=None):
        _check(lib().cs_graph_launch(ctypes.c_void_p(self.handle), _stream(stream)))

    def close(self):
        if self.handle:
            _check(lib().cs_graph_destroy(ctypes.c_void_p(self.handle)))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A batch of 3D patches.  patches: list of (u, b, tmp, stencil, h, parity)
    with caller-owned tensors (tmp with u's layout)."""

    def __init__(self, patches):
        self.patches = list(patches)
        descs = [describe(u, dim=3, stencil=st, h=h, parity=par) for (u, b, t, st, h, par) in self.patches]
        for (u, b, t, st, h, par) in self.patches:
            if u.shape != b.shape or u.stride() != b.stride() or t.shape != u.shape or t.stride() != u.stride():
                raise ValueError("u, b and tmp of a patch must share shape and strides")
        self.handle = cs_batch_create(descs, [p[0].data_ptr() for p in self.patches],
                                      [p[1].data_ptr() for p in self.patches],
                                      [p[2].data_ptr() for p in self.patches])
        self.norms = torch.zeros(len(self.patches), 3, dtype=torch.float64,
                                 device=self.patches[0][0].device)

    def close(self):
        if self.handle:
            cs_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def gs(self, nsweeps, stream=None):
        cs_batch_gs_sweeps(self.handle, nsweeps, stream)

    def sweeps_per_pass(self, index):
        return cs_batch_sweeps_per_pass(self.handle, index)

    def residual(self, stream=None):
        cs_batch_residual(self.handle, self.norms.data_ptr(), stream)
        return self.norms
