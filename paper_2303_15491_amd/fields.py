"""Seeded synthetic scalar fields for the segmentation workloads.

This module only draws inputs.  It holds none of the segmentation's
arithmetic, so it can feed both the GPU library and the CPU oracle the same
bits.  Fields are drawn in float64 with numpy's PCG64 generator and then cast
to float32 (or kept as float64).  Layout is C-contiguous ``(nz, ny, nx)``
(``(ny, nx)`` in 2-D), so vertex id ``v = x + nx*(y + ny*z)`` is the flat
index.

The workloads stand in for the paper's datasets (Noisy Terrain, Foot CT,
Rayleigh-Taylor "Miranda"), which are not used: only their shapes are kept.

* ``gaussian_mix_2d``  -- 64x64 sum of 8 isotropic Gaussians plus uniform noise.
* ``smoothed_noise``   -- white noise N(0,1) Gaussian-smoothed (separable,
  normalised kernel, truncated at 4 sigma, reflecting boundary), plus an
  optional linear ramp along z (256^3 at sigma 3, 512^3 at sigma 1.5).
* ``gaussian_blobs``   -- 3-D sum of 16..256 random Gaussians plus N(0, 0.02)
  noise, one member of the uneven batch.
* ``batch_shapes`` / ``batch_fields`` -- the 64-field uneven batch.
* ``serving_trace``    -- Poisson arrivals of mixed 2-D and 3-D requests.
* ``random_labels``    -- int32 labels drawn uniformly from {0..k-1}.
* ``region_labels``    -- piecewise-constant int32 labels of warped boxes with
  salt, the shape of a segmentation's label field (inputs of the marching
  index at sizes the oracle cannot segment in a test).
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_mix_2d(n: int = 64, count: int = 8, seed: int = 1, dtype=np.float32) -> np.ndarray:
    """Sum of ``count`` Gaussians a*exp(-|p-c|^2 / (2 s^2)) on an n x n grid,
    c ~ U[0, n-1]^2, s ~ U[3, 10], a ~ U[-1, 1], plus U[-0.01, 0.01] noise."""
    rng = _rng(seed)
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    f = np.zeros((n, n), np.float64)
    for _ in range(count):
        cx, cy = rng.uniform(0, n - 1, size=2)
        s = rng.uniform(3, 10)
        a = rng.uniform(-1, 1)
        f += a * np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2 * s * s))
    f += rng.uniform(-0.01, 0.01, size=(n, n))
    return f.astype(dtype)


def _smooth(a: np.ndarray, sigma: float) -> np.ndarray:
    from scipy.ndimage import gaussian_filter

    return gaussian_filter(a, sigma, mode="reflect", truncate=4.0)


def smoothed_noise(shape, sigma: float, seed: int, ramp: float = 0.0, dtype=np.float32) -> np.ndarray:
    """N(0,1) white noise smoothed with a Gaussian of std ``sigma`` voxels, plus
    ``ramp * z / (nz - 1)`` along the slowest axis.  Generated in float64, then
    cast."""
    rng = _rng(seed)
    a = rng.standard_normal(tuple(shape))
    a = _smooth(a, sigma)
    if ramp and a.ndim == 3 and a.shape[0] > 1:
        z = np.arange(a.shape[0], dtype=np.float64) / (a.shape[0] - 1)
        a += ramp * z[:, None, None]
    return a.astype(dtype, copy=False)


def gaussian_blobs(shape, seed: int, count=None, dtype=np.float32) -> np.ndarray:
    """Sum of 16..256 Gaussians (centre uniform in the box, s ~ U[2, 12],
    a ~ U[-1, 1]), each evaluated on the box of radius 4 s around its centre,
    plus N(0, 0.02) noise."""
    rng = _rng(seed)
    nz, ny, nx = shape
    if count is None:
        count = int(rng.integers(16, 257))
    f = np.zeros(shape, np.float64)
    for _ in range(count):
        c = rng.uniform([0, 0, 0], [nz - 1, ny - 1, nx - 1])
        s = rng.uniform(2, 12)
        a = rng.uniform(-1, 1)
        r = 4 * s
        sl, g = [], []
        for ax, n in enumerate(shape):
            lo, hi = max(0, int(np.floor(c[ax] - r))), min(n, int(np.ceil(c[ax] + r)) + 1)
            t = np.arange(lo, hi, dtype=np.float64)
            sl.append(slice(lo, hi))
            g.append(np.exp(-((t - c[ax]) ** 2) / (2 * s * s)))
        f[sl[0], sl[1], sl[2]] += a * g[0][:, None, None] * g[1][None, :, None] * g[2][None, None, :]
    f += rng.normal(0.0, 0.02, size=shape)
    return f.astype(dtype)


def batch_shapes(count: int = 64, seed: int = 4, lo: int = 32, hi: int = 192):
    """Per-axis sizes drawn uniformly from {lo..hi} for each batch member."""
    rng = _rng(seed)
    return [tuple(int(s) for s in rng.integers(lo, hi + 1, size=3)) for _ in range(count)]


def batch_fields(count: int = 64, seed: int = 4, lo: int = 32, hi: int = 192, dtype=np.float32):
    """The uneven batch: member j has shape ``batch_shapes(...)[j]`` and seed
    ``seed + j``."""
    return [gaussian_blobs(s, seed + j, dtype=dtype) for j, s in enumerate(batch_shapes(count, seed, lo, hi))]


def serving_trace(count: int, seed: int = 5, rate: float = 200.0):
    """Request descriptors for the serving workload: Poisson arrivals at
    ``rate`` per second; half 2-D n^2 fields (n in {128..2048}), half 3-D n^3
    fields (n in {64..384}); each smoothed N(0,1) noise with sigma in
    [1.5, 4] and its own seed.  Returns a list of dicts with keys ``t``
    (arrival time, s), ``shape``, ``sigma`` and ``seed``."""
    rng = _rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        if rng.random() < 0.5:
            n = int(rng.integers(128, 2049))
            shape = (n, n)
        else:
            n = int(rng.integers(64, 385))
            shape = (n, n, n)
        out.append({"t": t, "shape": shape, "sigma": float(rng.uniform(1.5, 4.0)),
                    "seed": int(rng.integers(0, 2**31 - 1))})
    return out


def random_labels(shape, k: int, seed: int) -> np.ndarray:
    """int32 labels drawn uniformly from {0..k-1} (PCG64)."""
    return _rng(seed).integers(0, k, size=tuple(shape), dtype=np.int32)


def region_labels(shape, seed: int, cell: float = 6.0, warp: float = 2.5, salt: float = 1e-3) -> np.ndarray:
    """Piecewise-constant int32 labels: each vertex takes the id of the box of
    side ``cell`` that holds it after every coordinate is shifted by a smooth
    warp of the other coordinates (warp * sin(2 pi (f1 u / n_u + f2 v / n_v) +
    phase), f ~ U{1..3}), so that region boundaries are curved surfaces; box
    ids are hashed to spread them over [0, 2^31).  Then a fraction ``salt`` of
    the vertices (drawn with repetition) get ids of their own, which adds
    cells with three and four labels."""
    rng = _rng(seed)
    shape = tuple(int(s) for s in shape)
    nd = len(shape)
    key = np.zeros(shape, np.uint32)
    for a in range(nd):
        others = [b for b in range(nd) if b != a]
        w = np.zeros([shape[b] if b != a else 1 for b in range(nd)], np.float32)
        if others:
            f = rng.integers(1, 4, size=len(others))
            phase = rng.uniform(0, 2 * np.pi)
            arg = np.full(w.shape, phase, np.float64)
            for fb, b in zip(f, others):
                t = np.arange(shape[b], dtype=np.float64) * (2 * np.pi * fb / shape[b])
                arg = arg + t.reshape([shape[b] if c == b else 1 for c in range(nd)])
            w = (warp * np.sin(arg)).astype(np.float32)
        c = np.arange(shape[a], dtype=np.float32).reshape([shape[a] if b == a else 1 for b in range(nd)])
        q = np.floor((c + w) / np.float32(cell)).astype(np.int32) + 16
        key *= np.uint32(1000003)
        key += q.astype(np.uint32)
    key *= np.uint32(2654435761)
    lab = (key >> np.uint32(1)).astype(np.int32)
    n = lab.size
    m = int(salt * n)
    if m:
        idx = rng.integers(0, n, size=m)
        lab.reshape(-1)[idx] = rng.integers(0, 2**31 - 1, size=m, dtype=np.int32)
    return lab


# The named workloads.
def workload_c1():
    """2-D 64x64 sum of Gaussians (seed 1)."""
    return gaussian_mix_2d(64, 8, seed=1)


def workload_c2(n: int = 256):
    """3-D n^3 noise smoothed at sigma 3 plus a 0.1 ramp along z (seed 2)."""
    return smoothed_noise((n, n, n), 3.0, seed=2, ramp=0.1)


def workload_c3(n: int = 512):
    """3-D n^3 noise smoothed at sigma 1.5 (seed 3); float32."""
    return smoothed_noise((n, n, n), 1.5, seed=3)


def serving_pool(count: int = 64, seed: int = 5, sigmas=(1.5, 2.75, 4.0), max3d: int = 384, max2d: int = 2048):
    """Host fields for the serving workload: ``count`` requests whose sizes
    follow ``serving_trace(count, seed)``, each cut (at a seeded offset) from
    one of a few smoothed-noise base fields -- the one whose sigma is nearest
    the request's.  Crops of smoothed noise are smoothed noise, and cutting is
    far cheaper than smoothing every request."""
    trace = serving_trace(count, seed=seed)
    rng = _rng(seed + 1)
    base3 = {s: smoothed_noise((max3d,) * 3, s, seed=seed * 100 + i) for i, s in enumerate(sigmas)}
    base2 = {s: smoothed_noise((max2d,) * 2, s, seed=seed * 100 + 50 + i) for i, s in enumerate(sigmas)}
    out = []
    for req in trace:
        sig = min(sigmas, key=lambda s: abs(s - req["sigma"]))
        base = base3[sig] if len(req["shape"]) == 3 else base2[sig]
        sl = []
        for n, m in zip(req["shape"], base.shape):
            n = min(n, m)  # a request larger than the base is cut to the base
            o = int(rng.integers(0, m - n + 1))
            sl.append(slice(o, o + n))
        out.append(np.ascontiguousarray(base[tuple(sl)]))
    return trace, out
