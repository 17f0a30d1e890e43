"""The allocation-free residual entry point against cs_residual, through the
C ABI: the same r and the same norms, bit for bit, on two calls in a row (the
second on a smaller grid, reusing the device's fixed scratch), in 3D and 2D,
FP64 and FP32, and on a plane too large for the streaming residual."""
import numpy as np
import pytest
import torch

from paper_1810_04033_amd import colsten as C

import gpu_util as G

pytestmark = pytest.mark.gpu


def _both(dim, n, st, seed, dtype=torch.float64):
    u, b = G.case(dim, n, seed=seed)
    h = 1.0 / (max(n) + 1)
    ug, bg = G.upload(u, dtype), G.upload(b, dtype)
    r_ref, r_new = C.grid_like(ug), C.grid_like(ug)
    r_new.fill_(7.0)
    g = C.Grid(ug, bg, dim=dim, stencil=st, h=h)
    want = g.residual(r=r_ref).clone()
    g.close()
    d = C.describe(ug, dim=dim, stencil=st, h=h)
    got = torch.full((3,), -1.0, dtype=torch.float64, device="cuda")
    C.cs_residual_noalloc(d, ug.data_ptr(), bg.data_ptr(), r_new.data_ptr(), got.data_ptr())
    only_norms = torch.full((3,), -1.0, dtype=torch.float64, device="cuda")
    C.cs_residual_noalloc(d, ug.data_ptr(), bg.data_ptr(), 0, only_norms.data_ptr())
    torch.cuda.synchronize()
    return want.cpu().numpy(), got.cpu().numpy(), only_norms.cpu().numpy(), r_ref, r_new


@pytest.mark.parametrize("first,second", [
    ((3, (96, 80, 40), C.CS_FD), (3, (17, 9, 5), C.CS_Q1)),
    ((3, (70, 33, 21), C.CS_Q1), (2, (31, 12), C.CS_FD)),
    ((2, (300, 200), C.CS_Q1), (3, (5, 4, 3), C.CS_FD)),
])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_residual_equals_cs_residual(first, second, dtype):
    for seed, (dim, n, st) in ((900, first), (901, second)):
        want, got, only, r_ref, r_new = _both(dim, n, st, seed, dtype)
        assert np.array_equal(got, want)
        assert np.array_equal(only, want)
        assert torch.equal(r_new[(slice(1, -1),) * dim], r_ref[(slice(1, -1),) * dim])


def test_noalloc_residual_on_planes_beyond_the_streaming_grid():
    for seed, n in ((910, (1100, 1100, 3)), (911, (40, 30, 20))):
        want, got, only, r_ref, r_new = _both(3, n, C.CS_Q1, seed)
        assert np.array_equal(got, want)
        assert torch.equal(r_new[1:-1, 1:-1, 1:-1], r_ref[1:-1, 1:-1, 1:-1])


def test_noalloc_residual_rejects_bad_arguments():
    u, b = G.case(3, (8, 8, 8), seed=920)
    ug, bg = G.upload(u), G.upload(b)
    d = C.describe(ug, dim=3, stencil=C.CS_FD, h=1.0 / 9)
    norms = torch.zeros(3, dtype=torch.float64, device="cuda")
    with pytest.raises(C.ColstenError):
        C.cs_residual_noalloc(d, ug.data_ptr(), bg.data_ptr(), 0, 0)  # neither r nor norms
    with pytest.raises(C.ColstenError):
        C.cs_residual_noalloc(d, ug.data_ptr(), ug.data_ptr(), 0, norms.data_ptr())  # u == b
    with pytest.raises(C.ColstenError):
        C.cs_residual_noalloc(d, ug.data_ptr(), bg.data_ptr(), ug.data_ptr(), norms.data_ptr())
    with pytest.raises(C.ColstenError):  # b not aligned to its element size
        C.cs_residual_noalloc(d, ug.data_ptr(), bg.data_ptr() + 4, 0, norms.data_ptr())
    d.dim = 4
    with pytest.raises(C.ColstenError):
        C.cs_residual_noalloc(d, ug.data_ptr(), bg.data_ptr(), 0, norms.data_ptr())
