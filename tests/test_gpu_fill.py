"""The device-side seeded fill against the host-side input generator: the same
SplitMix64 counter stream, so the fields must agree bit for bit (FP64; FP32 is
the FP64 value rounded), on every layout, with the halo left untouched."""
import numpy as np
import pytest
import torch

from paper_1810_04033_amd import colsten as C
from paper_1810_04033_amd import inputs as I

import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim,n", [(2, (1, 1)), (2, (37, 21)), (3, (17, 9, 12)), (3, (65, 14, 5))],
                         ids=lambda p: "x".join(map(str, p)) if isinstance(p, tuple) else str(p))
@pytest.mark.parametrize("dt", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("layout", ["aligned", "compact", "odd"])
def test_fill_matches_host_generator(dim, n, dt, layout):
    seed = I.stream_seed(77, 3)
    shape = tuple(reversed(n))
    sentinel = np.full(tuple(s + 2 for s in shape), 7.25)
    t = G.upload(sentinel, dt, layout=layout)
    C.fill_uniform(t, seed, dim=dim)
    torch.cuda.synchronize()
    got = t.detach().cpu().numpy()
    want = I.uniform_field(seed, shape).astype(got.dtype)
    inner = (slice(1, -1),) * dim
    assert np.array_equal(got[inner], want)
    mask = np.ones(got.shape, dtype=bool)
    mask[inner] = False
    assert np.all(got[mask] == np.float64(7.25).astype(got.dtype))


def test_fill_rejects_null_and_host_pointers():
    t = C.empty_grid((5, 4), dtype=torch.float64)
    d = C.describe(t, dim=2, stencil=C.CS_FD, h=1.0)
    host = np.zeros(t.numel())
    for ptr in (None, host.ctypes.data):
        st = C.lib().cs_fill_uniform(C.ctypes.byref(d), C.ctypes.c_void_p(ptr), C.ctypes.c_uint64(1), None)
        assert st == C.CS_EINVAL
    # The range check covers the HIP allocation holding the pointer, which for
    # torch's caching allocator is a segment of 2 MiB or more: overrun it.
    big = C.empty_grid((2048, 2048), dtype=torch.float64)
    dbig = C.describe(big, dim=2, stencil=C.CS_FD, h=1.0)
    st = C.lib().cs_fill_uniform(C.ctypes.byref(dbig), C.ctypes.c_void_p(t.data_ptr()), C.ctypes.c_uint64(1), None)
    assert st == C.CS_EINVAL
