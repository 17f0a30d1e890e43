"""Seeded synthetic inputs for the coloured stencil sweeps.

This module is the one piece shared by the GPU path and the oracle: it only
draws numbers and lays them out.  It contains none of the method's arithmetic
(no stencil, sweep, residual or norm).

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used in counter form:

    value(seed, l) = mix64(seed + (l + 1) * 0x9E3779B97F4A7C15)   (mod 2^64)

which equals the l-th output (0-based) of the sequential generator started at
state ``seed``.  ``l`` is the 0-based lexicographic interior index with x
fastest, so a field does not depend on the array layout (padding, halo).
Uniform[-1, 1) is ``(v >> 11) * 2^-52 - 1``, exact in binary64.  Independent
streams use ``seed' = mix64(seed ^ stream)``.

Workload recipes (the shapes and distributions of the benchmark configurations):

* ``uniform_rhs``: i.i.d. uniform[-1, 1) right-hand side on an n^d grid.
* ``fourier_rhs``: a sum of random low Fourier modes with N(0,1) amplitudes
  (Box-Muller) plus uniform[-1e-3, 1e-3] point noise.
* ``patch_edges``: cubic patch edge lengths drawn uniformly from a list.
* ``request_stream``: Poisson arrivals of patch solves with log-uniform edges,
  bounded aspect ratio, and a stencil/precision mix.
"""
from dataclasses import dataclass

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mix64(z):
    """SplitMix64 output mixer on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed, index):
    """value(seed, l) for an array of counters l (uint64)."""
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (idx + np.uint64(1)) * GAMMA
    return mix64(z)


def stream_seed(seed, stream):
    """Seed of an independent stream: mix64(seed ^ stream)."""
    return int(mix64(np.uint64(seed) ^ np.uint64(stream)))


def u01(v):
    """uniform [0, 1) doubles from uint64 draws (53 high bits)."""
    return (np.asarray(v, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def uniform_pm1(v):
    """uniform [-1, 1) doubles from uint64 draws; exact in binary64."""
    return (np.asarray(v, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0


def uniform_field(seed, shape_zyx):
    """An interior field of shape (nz, ny, nx) or (ny, nx) of uniform[-1,1)."""
    count = int(np.prod(shape_zyx))
    out = np.empty(count, dtype=np.float64)
    chunk = 1 << 24
    for s in range(0, count, chunk):
        e = min(count, s + chunk)
        out[s:e] = uniform_pm1(splitmix64(seed, np.arange(s, e, dtype=np.uint64)))
    return out.reshape(shape_zyx)


def fourier_field(seed, n, modes=32, max_freq=32, noise=1e-3):
    """sum_m a_m sin(pi p_m x) sin(pi q_m y) sin(pi r_m z) + eta on the
    interior points x = i h, i = 1..n, h = 1/(n+1) (3D, shape (n, n, n)).
    p, q, r uniform in {1..max_freq}; a_m ~ N(0,1) by Box-Muller; eta uniform
    in [-noise, noise).  Uses libm sin through numpy."""
    ms = stream_seed(seed, 1)
    draws = splitmix64(ms, np.arange(5 * modes, dtype=np.uint64)).reshape(modes, 5)
    freq = (draws[:, :3] % np.uint64(max_freq)).astype(np.int64) + 1
    u1 = 1.0 - u01(draws[:, 3])  # (0, 1]
    u2 = u01(draws[:, 4])
    amp = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1, dtype=np.float64) * h
    out = np.zeros((n, n, n), dtype=np.float64)
    for m in range(modes):
        sx = np.sin(np.pi * freq[m, 0] * x)
        sy = np.sin(np.pi * freq[m, 1] * x)
        sz = np.sin(np.pi * freq[m, 2] * x)
        plane = amp[m] * np.outer(sy, sx)
        for k in range(n):
            out[k] += sz[k] * plane
    out += noise * uniform_field(stream_seed(seed, 2), (n, n, n))
    return out


def halo_array(interior, pitch=None, dtype=np.float64, halo_value=0.0):
    """Embed an interior field in a halo'd array with row pitch >= nx + 2.

    Returns the halo'd view (shape (nz+2, ny+2, nx+2) or (ny+2, nx+2)); when a
    pitch is given the view's rows are padded (the padding is zero)."""
    interior = np.asarray(interior)
    shp = tuple(s + 2 for s in interior.shape)
    px = shp[-1] if pitch is None else int(pitch)
    if px < shp[-1]:
        raise ValueError("pitch must be at least nx + 2")
    full = np.zeros(shp[:-1] + (px,), dtype=dtype)
    view = full[..., :shp[-1]]
    view[...] = halo_value
    view[(slice(1, -1),) * interior.ndim] = interior
    return view


def patch_edges(seed, count, choices=(8, 16, 24, 32, 48, 64)):
    """Edge lengths of `count` cubic patches, uniform over `choices`."""
    v = splitmix64(seed, np.arange(count, dtype=np.uint64))
    return [int(choices[int(x % np.uint64(len(choices)))]) for x in v]


@dataclass
class Request:
    rid: int
    arrival_s: float
    n: tuple          # (nx, ny, nz)
    stencil: int      # 0 = 7-point, 1 = 27-point
    mixed: bool       # True = FP32 sweeps inside FP64 refinement
    rhs_seed: int


def request_stream(seed, count, rate_per_s, edge_lo=16, edge_hi=128, max_aspect=4.0):
    """Poisson arrivals (exponential gaps, mean 1/rate) of 3D patch solves.

    Each axis length is round(edge_lo * (edge_hi/edge_lo)**U) (log-uniform);
    a triple with max/min > max_aspect is redrawn.  Stencil and precision are
    each a fair coin.  The RHS of request i uses stream seed (seed, 1000 + i)."""
    out = []
    t = 0.0
    ctr = 0
    base = stream_seed(seed, 7)
    ratio = edge_hi / edge_lo

    def nxt():
        nonlocal ctr
        v = splitmix64(base, np.array([ctr], dtype=np.uint64))[0]
        ctr += 1
        return float(u01(v))

    for i in range(count):
        t += -np.log(1.0 - nxt()) / rate_per_s
        while True:
            n = tuple(int(round(edge_lo * ratio ** nxt())) for _ in range(3))
            if max(n) / min(n) <= max_aspect:
                break
        stencil = 0 if nxt() < 0.5 else 1
        mixed = nxt() >= 0.5
        out.append(Request(i, t, n, stencil, mixed, stream_seed(seed, 1000 + i)))
    return out
