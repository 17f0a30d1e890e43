"""Helpers of the GPU tests: seeded cases, upload with chosen layouts, compare."""
import numpy as np
import torch

from paper_1810_04033_amd import inputs as I
from paper_1810_04033_amd import colsten as C


def case(dim, n, seed, halo=True):
    """(u0, b) compact halo'd float64 arrays: random interior, random halo."""
    shape = tuple(reversed(n[:dim]))
    u = I.halo_array(I.uniform_field(I.stream_seed(seed, 1), shape))
    b = I.halo_array(I.uniform_field(I.stream_seed(seed, 2), shape))
    if halo:
        full = I.uniform_field(I.stream_seed(seed, 3), u.shape)
        mask = np.ones(u.shape, dtype=bool)
        mask[(slice(1, -1),) * dim] = False
        u[mask] = 0.5 * full[mask]
    return u, b


def upload(a, dtype=torch.float64, layout="aligned"):
    """Copy a compact halo'd numpy array to the GPU in the given layout:
    'aligned' (128-byte rows), 'compact', or 'odd' (odd pitch, odd offset)."""
    n = tuple(reversed([s - 2 for s in a.shape]))
    if layout == "aligned":
        t = C.empty_grid(n, dtype=dtype)
    elif layout == "compact":
        t = torch.zeros(a.shape, dtype=dtype, device="cuda")
    else:
        px = a.shape[-1] + 3
        rows = int(np.prod(a.shape[:-1]))
        flat = torch.zeros(5 + rows * px + 7, dtype=dtype, device="cuda")
        strides = []
        acc = px
        for v in reversed(a.shape[:-1]):
            strides.insert(0, acc)
            acc *= v
        t = flat.as_strided(a.shape, tuple(strides) + (1,), storage_offset=5)
    t.copy_(torch.from_numpy(a).to(dtype))
    return t


def download(t):
    return t.detach().cpu().numpy().astype(np.float64)


def relmax(a, b):
    den = max(float(np.max(np.abs(b))), 1e-300)
    return float(np.max(np.abs(np.asarray(a, dtype=np.float64) - b))) / den
