"""Argument validation and ownership through the C ABI (on a GPU).

Every bad call must come back with a status and a message before anything is
launched; none of these tests launches a kernel on invalid memory."""
import numpy as np
import pytest
import torch

from paper_1810_04033_amd import colsten as C

pytestmark = pytest.mark.gpu


def _grid(n=(8, 6, 5), dtype=torch.float64):
    u = C.empty_grid(n, dtype=dtype)
    b = C.empty_grid(n, dtype=dtype)
    return u, b


def _expect(status, fn, *args):
    with pytest.raises(C.ColstenError) as ei:
        fn(*args)
    assert ei.value.status == status
    assert C.cs_last_error()


def test_bad_descriptors():
    u, b = _grid()
    for field, value in (("dim", 4), ("stencil", 7), ("dtype", 9), ("parity", 2)):
        d = C.describe(u, dim=3, stencil=C.CS_FD, h=0.1)
        setattr(d, field, value)
        _expect(C.CS_EINVAL, C.cs_grid_create, d, u.data_ptr(), b.data_ptr())
    d = C.describe(u, dim=3, stencil=C.CS_FD, h=0.1)
    d.n[0] = 0
    _expect(C.CS_EINVAL, C.cs_grid_create, d, u.data_ptr(), b.data_ptr())
    d = C.describe(u, dim=3, stencil=C.CS_FD, h=0.1)
    d.stride[0] = 2
    _expect(C.CS_EINVAL, C.cs_grid_create, d, u.data_ptr(), b.data_ptr())
    d = C.describe(u, dim=3, stencil=C.CS_FD, h=-1.0)
    _expect(C.CS_EINVAL, C.cs_grid_create, d, u.data_ptr(), b.data_ptr())
    d = C.describe(u, dim=3, stencil=C.CS_FD, h=float("nan"))
    _expect(C.CS_EINVAL, C.cs_grid_create, d, u.data_ptr(), b.data_ptr())


def test_bad_pointers():
    u, b = _grid()
    d = C.describe(u, dim=3, stencil=C.CS_Q1, h=0.1)
    _expect(C.CS_EINVAL, C.cs_grid_create, d, 0, b.data_ptr())
    host = np.zeros(4096)
    _expect(C.CS_EINVAL, C.cs_grid_create, d, host.ctypes.data, b.data_ptr())
    _expect(C.CS_EINVAL, C.cs_grid_create, d, u.data_ptr(), u.data_ptr())
    # a descriptor far larger than the allocation is refused before any launch
    big = C.describe(u, dim=3, stencil=C.CS_Q1, h=0.1)
    big.n[2] = 100000
    big.stride[2] = big.stride[1] * (big.n[1] + 2)
    _expect(C.CS_EINVAL, C.cs_grid_create, big, u.data_ptr(), b.data_ptr())


def test_bad_calls_on_a_valid_grid():
    u, b = _grid()
    g = C.Grid(u, b, dim=3, stencil=C.CS_Q1, h=0.1)
    _expect(C.CS_EINVAL, C.cs_colour_pass, g.handle, 8)
    _expect(C.CS_EINVAL, C.cs_colour_pass, g.handle, -1)
    _expect(C.CS_EINVAL, C.cs_gs_sweeps, g.handle, -1, 0)
    _expect(C.CS_EINVAL, C.cs_jacobi_sweeps, g.handle, 0.5, 1, 0)
    _expect(C.CS_EINVAL, C.cs_jacobi_sweeps, g.handle, float("inf"), 1, C.grid_like(u).data_ptr())
    _expect(C.CS_EINVAL, C.cs_gs_sweeps, g.handle, 2, u.data_ptr())
    _expect(C.CS_EINVAL, C.cs_residual, g.handle, 0, 0)
    g.close()


def test_zero_sweeps_and_destroy_leave_buffers_alone():
    u, b = _grid()
    u.normal_()
    ref = u.clone()
    g = C.Grid(u, b, dim=3, stencil=C.CS_FD, h=0.1)
    g.gs(0)
    g.close()
    C.cs_grid_destroy(0)
    torch.cuda.synchronize()
    assert torch.equal(u, ref)


def test_num_colours():
    for dim, st, want in ((2, C.CS_FD, 2), (3, C.CS_FD, 2), (2, C.CS_Q1, 4), (3, C.CS_Q1, 8)):
        n = (4, 4, 4)[:dim]
        u, b = _grid(n)
        g = C.Grid(u, b, dim=dim, stencil=st, h=0.2)
        assert g.num_colours == want
        g.close()
