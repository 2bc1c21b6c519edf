"""Seeded synthetic scalar fields shaped like the paper's workloads.

The paper measures on real simulation outputs (its Table II: 2D/3D, float32
and float64, 4 MB to 1.13 GB) that are not available here; these generators
stand in for them.  Every field is produced on the host with numpy's PCG64
generator in float64 and then rounded to the target dtype, so the same seed
gives the same bytes on the same machine.  Transcendental functions in numpy
may differ in the last bit between CPUs, so expected values are always
recomputed on the machine that runs the comparison.

This module holds no compression arithmetic: it only makes inputs.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

__all__ = [
    "gaussian_bumps", "power_law_grf", "smooth_field", "turbulence_field",
    "lognormal_field", "fronts_field", "batch_fields", "serving_requests",
    "reflect_tile", "CONFIGS",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_bumps(shape, seed: int = 0, n_bumps: int = 32, noise: float = 1e-3,
                   dtype=np.float32, sigma_range=(8.0, 64.0)) -> np.ndarray:
    """Sum of ``n_bumps`` random anisotropic Gaussians plus white noise.

    2D: amplitude U[-1,1], two axis widths U[sigma_range] px, rotation U[0,pi),
    centre uniform over the grid.  3D: the same with three axis widths and a
    random rotation (from a QR factorisation of a Gaussian matrix).  Noise is
    i.i.d. N(0, noise^2).
    """
    rng = _rng(seed)
    shape = tuple(int(s) for s in shape)
    nd = len(shape)
    bumps = []
    for _ in range(n_bumps):
        amp = rng.uniform(-1.0, 1.0)
        sig = rng.uniform(sigma_range[0], sigma_range[1], size=nd)
        centre = np.array([rng.uniform(0, s) for s in shape])
        if nd == 2:
            th = rng.uniform(0.0, math.pi)
            rot = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
        else:
            q, r = np.linalg.qr(rng.standard_normal((3, 3)))
            rot = q * np.sign(np.diag(r))
        bumps.append((amp, centre, rot @ np.diag(1.0 / sig ** 2) @ rot.T))
    out = np.zeros(shape, np.float64)

    def slab(lo, hi):
        # the quadratic form split into terms over pairs of axes, so that only
        # their sum runs over the full grid
        sub = out[lo:hi]
        axes = [np.arange(lo, hi, dtype=np.float64)] + \
            [np.arange(s, dtype=np.float64) for s in shape[1:]]
        grids = np.meshgrid(*axes, indexing="ij", sparse=True)
        for amp, centre, P in bumps:
            d = [g - c for g, c in zip(grids, centre)]
            if nd == 2:
                quad = P[0, 0] * (d[0] * d[0]) + (P[0, 1] + P[1, 0]) * (d[0] * d[1]) + \
                    P[1, 1] * (d[1] * d[1])
            else:
                a = P[0, 0] * (d[0] * d[0]) + (P[0, 1] + P[1, 0]) * (d[0] * d[1]) + \
                    P[1, 1] * (d[1] * d[1])
                b = (P[0, 2] + P[2, 0]) * (d[0] * d[2])
                c = (P[1, 2] + P[2, 1]) * (d[1] * d[2]) + P[2, 2] * (d[2] * d[2])
                quad = a + b
                quad += c
            np.multiply(quad, -0.5, out=quad)
            np.exp(quad, out=quad)
            quad *= amp
            sub += quad

    # slabs of about 256K points keep the temporaries small; numpy's
    # element-wise loops release the GIL, so slabs run on threads
    n0 = shape[0]
    plane = max(1, out.size // n0)
    step = max(1, (1 << 18) // plane)
    workers = max(1, min(16, os.cpu_count() or 1))
    if workers == 1 or n0 <= step:
        slab(0, n0)
    else:
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(lambda lo: slab(lo, min(n0, lo + step)), range(0, n0, step)))
    if noise:
        out += rng.normal(0.0, noise, size=shape)
    return out.astype(dtype)


def power_law_grf(shape, slope: float, seed: int = 0) -> np.ndarray:
    """Gaussian random field with power spectrum P(k) ~ |k|^-slope (k = 0
    removed), standardised to zero mean and unit variance (float64)."""
    rng = _rng(seed)
    shape = tuple(int(s) for s in shape)
    white = rng.standard_normal(shape)
    spec = np.fft.rfftn(white)
    ks = [np.fft.fftfreq(s) for s in shape[:-1]] + [np.fft.rfftfreq(shape[-1])]
    k2 = np.zeros(spec.shape, np.float64)
    for a, k in enumerate(ks):
        sh = [1] * len(shape)
        sh[a] = k.size
        k2 = k2 + (k.reshape(sh) ** 2)
    amp = np.zeros_like(k2)
    nz = k2 > 0
    amp[nz] = k2[nz] ** (-slope / 4.0)  # |k|^(-slope/2) on the amplitude
    spec *= amp
    del k2, amp
    g = np.fft.irfftn(spec, s=shape, axes=tuple(range(len(shape))))
    g -= g.mean()
    g /= g.std()
    return g


def smooth_field(shape=(512, 512), seed: int = 0, dtype=np.float32) -> np.ndarray:
    """2D float32 512x512 workload: 32 anisotropic Gaussians + N(0, 1e-3)."""
    return gaussian_bumps(shape, seed=seed, n_bumps=32, noise=1e-3, dtype=dtype)


def turbulence_field(shape=(256, 256, 256), seed: int = 0, dtype=np.float32) -> np.ndarray:
    """3D float32 256^3 workload: power-law GRF with P(k) ~ k^-3, plus 1%
    white noise (std 0.01 relative to the standardised field), min-max
    normalised to [0, 1]."""
    g = power_law_grf(shape, 3.0, seed)
    g += 0.01 * _rng(seed + 7_000_001).standard_normal(g.shape)
    g -= g.min()
    g /= g.max()
    return g.astype(dtype)


def lognormal_field(shape=(512, 512, 512), seed: int = 0, dtype=np.float64) -> np.ndarray:
    """3D float64 512^3 workload: exp(2 g) of a k^-2.5 GRF g, floored at its
    10th percentile so that about a tenth of the points form exact-tie
    plateaus; heavy tailed, most points in the lowest bins."""
    g = power_law_grf(shape, 2.5, seed)
    np.multiply(g, 2.0, out=g)
    np.exp(g, out=g)
    floor = np.partition(g.ravel(), g.size // 10)[g.size // 10]
    np.maximum(g, floor, out=g)
    return g.astype(dtype, copy=False)


def fronts_field(shape=(1800, 3600), seed: int = 0, dtype=np.float32) -> np.ndarray:
    """2D float32 1800x3600 workload, periodic on both axes: 8 sinusoidal
    modes plus 4 sharp tanh fronts (width 1-4 px) along smooth periodic
    level sets."""
    rng = _rng(seed)
    n0, n1 = int(shape[0]), int(shape[1])
    i = np.arange(n0, dtype=np.float64)[:, None] / n0
    j = np.arange(n1, dtype=np.float64)[None, :] / n1
    out = np.zeros((n0, n1), np.float64)
    for _ in range(8):
        a, b = rng.integers(1, 7, size=2)
        amp = rng.uniform(0.2, 1.0)
        ph = rng.uniform(0, 2 * math.pi)
        out += amp * np.sin(2 * math.pi * (a * i + b * j) + ph)
    for _ in range(4):
        amp = rng.uniform(0.5, 1.5)
        w = rng.uniform(1.0, 4.0)
        h = np.zeros((n0, n1), np.float64)
        for _ in range(2):
            a, b = rng.integers(1, 4, size=2)
            ph = rng.uniform(0, 2 * math.pi)
            h += rng.uniform(40.0, 120.0) * np.sin(2 * math.pi * (a * i + b * j) + ph)
        out += amp * np.tanh((h + rng.uniform(-20.0, 20.0)) / w)
    return out.astype(dtype)


def batch_fields(n_fields: int = 256, seed: int = 0, scale: float = 1.0):
    """Batched workload: ``n_fields`` fields of uneven size.  Each is 2D or 3D
    with probability 1/2; side length log-uniform in [64, 1024] (2D) or
    [32, 192] (3D), times ``scale``; content as the 2D Gaussian workload (3D
    Gaussians for 3D); per-field NOA bound log-uniform in [1e-4, 1e-2].
    Field i uses seed 1000 + i.  Returns a list of (field, eb)."""
    rng = _rng(seed)
    out = []
    for f in range(n_fields):
        three_d = rng.random() < 0.5
        lo, hi = (32, 192) if three_d else (64, 1024)
        side = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))) * scale))
        side = max(side, 2)
        eb = float(math.exp(rng.uniform(math.log(1e-4), math.log(1e-2))))
        shape = (side,) * (3 if three_d else 2)
        x = gaussian_bumps(shape, seed=1000 + f, n_bumps=32, noise=1e-3,
                           dtype=np.float32)
        out.append((x, eb))
    return out


def serving_requests(n: int, seed: int = 7, min_bytes: int = 1 << 20,
                     max_bytes: int = 512 << 20):
    """Serving workload descriptors: each request is a compress (p = 1/2) or
    decompress, dtype float32/float64 and 2D/3D uniform, size log-uniform in
    [min_bytes, max_bytes], NOA bound log-uniform in [1e-4, 1e-2].  Returns a
    list of dicts with keys op, dtype, shape, eb."""
    rng = _rng(seed)
    reqs = []
    for _ in range(n):
        op = "compress" if rng.random() < 0.5 else "decompress"
        dt = np.float32 if rng.random() < 0.5 else np.float64
        nd = 2 if rng.random() < 0.5 else 3
        nbytes = math.exp(rng.uniform(math.log(min_bytes), math.log(max_bytes)))
        pts = max(64, int(nbytes / np.dtype(dt).itemsize))
        if nd == 2:
            a = int(round(math.sqrt(pts)))
            shape = (a, max(1, pts // a))
        else:
            a = int(round(pts ** (1 / 3)))
            shape = (a, a, max(1, pts // (a * a)))
        eb = float(math.exp(rng.uniform(math.log(1e-4), math.log(1e-2))))
        reqs.append({"op": op, "dtype": dt, "shape": shape, "eb": eb})
    return reqs


def reflect_tile(base, shape):
    """A field of ``shape`` made from ``base`` (same number of axes) by
    mirror tiling: index i of an axis of length n reads base index
    r(i mod 2n) with r(j) = j for j < n, 2n - 1 - j otherwise.  Works on
    numpy arrays and on torch tensors (on their device), so serving payloads
    of any size come from a few generated fields."""
    idx = []
    for n, m in zip(base.shape, shape):
        j = np.arange(int(m)) % (2 * n)
        j = np.where(j < n, j, 2 * n - 1 - j)
        idx.append(j)
    if isinstance(base, np.ndarray):
        return np.ascontiguousarray(base[np.ix_(*idx)])
    import torch
    out = base
    for ax, j in enumerate(idx):
        out = torch.index_select(out, ax, torch.from_numpy(j).to(base.device))
    return out.contiguous()


#: The workloads by name: generator, full shape, NOA bounds.
CONFIGS = {
    "smooth2d": (smooth_field, (512, 512), (1e-3,)),
    "turb3d": (turbulence_field, (256, 256, 256), (1e-2, 1e-3, 1e-4)),
    "lognormal3d": (lognormal_field, (512, 512, 512), (1e-3,)),
    "fronts2d": (fronts_field, (1800, 3600), (1e-3,)),
}
