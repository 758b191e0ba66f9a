"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no stencil arithmetic: it only draws random numbers and
evaluates the closed-form initial fields of the five workloads, so both the
oracle side and the HIP side consume the identical rounded arrays.

Random streams: numpy PCG64 seeded with ``SeedSequence([workload_id, stream])``
(workload ids 1..5 as numbered below; stream ids per array).  Values are drawn
or evaluated in FP64 and rounded once to the run dtype.

Workloads (sizes are the full-size defaults; every generator also takes smaller
sizes for tests):
  1. 1D periodic, N = 2^20 fp64, r = 0.25, 100 steps; u0 = sum of sine modes
     k = 1, 7, 31, 127 (amplitude 1) + uniform[-1e-3, 1e-3] noise.
  2. 1D periodic, N = 2^28 fp32 split into 64 partitions of 4 Mi cells, r = 0.25,
     50 steps; u0 ~ uniform[0, 1].
  3. 4096 independent periodic problems, n log-uniform in [1024, 2^20], r ~
     uniform[0.05, 0.25], 20 steps, fp32; u0 ~ uniform[0, 1].
  4. 2D 16384 x 16384 fp32, zero-Dirichlet, r = 0.2, 200 steps, 16 row bands;
     u0 = 64 Gaussian bumps (sigma 200 cells), separable and truncated at 8 sigma.
  5. 2D 8192 x 8192 fp32 variable coefficient, dt = 0.2, 100 steps; kappa =
     min(exp(-2 + 0.5 z), 1), z ~ N(0, 1); u0 = 64 Gaussian bumps (sigma 100);
     target ~ uniform[0, 1].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def rng(workload_id: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([workload_id, stream])))


# ----------------------------------------------------------------- workload specs
@dataclass(frozen=True)
class Periodic1D:
    n: int = 1 << 20
    r: float = 0.25
    steps: int = 100
    modes: tuple = (1, 7, 31, 127)
    noise: float = 1e-3
    dtype: str = "f64"


@dataclass(frozen=True)
class Partitioned1D:
    n: int = 1 << 28
    parts: int = 64
    r: float = 0.25
    steps: int = 50
    dtype: str = "f32"


@dataclass(frozen=True)
class Batched1D:
    count: int = 4096
    nmin: int = 1024
    nmax: int = 1 << 20
    rmin: float = 0.05
    rmax: float = 0.25
    steps: int = 20
    dtype: str = "f32"


@dataclass(frozen=True)
class Banded2D:
    ny: int = 16384
    nx: int = 16384
    bands: int = 16
    r: float = 0.2
    steps: int = 200
    centres: int = 64
    sigma: float = 200.0
    dtype: str = "f32"


@dataclass(frozen=True)
class VarCoef2D:
    ny: int = 8192
    nx: int = 8192
    dt: float = 0.2
    steps: int = 100
    ckpt: int = 10
    mu: float = -2.0
    sigma_log: float = 0.5
    kappa_max: float = 1.0
    centres: int = 64
    sigma: float = 100.0
    dtype: str = "f32"


NP_DTYPE = {"f32": np.float32, "f64": np.float64}


# -------------------------------------------------------------------- generators
def sine_modes(n: int, modes) -> np.ndarray:
    """sum_k sin(2 pi k i / n), i = 0..n-1, in FP64."""
    i = np.arange(n, dtype=np.float64)
    u = np.zeros(n, dtype=np.float64)
    for k in modes:
        u += np.sin(2.0 * np.pi * float(k) * i / float(n))
    return u


def periodic1d_u0(spec: Periodic1D = Periodic1D(), with_noise: bool = True) -> np.ndarray:
    u = sine_modes(spec.n, spec.modes)
    if with_noise and spec.noise > 0:
        u = u + rng(1, 0).uniform(-spec.noise, spec.noise, spec.n)
    return u.astype(NP_DTYPE[spec.dtype])


def partitioned1d_u0(spec: Partitioned1D = Partitioned1D(), out=None) -> np.ndarray:
    """uniform[0, 1] of the run dtype; `out` may be a preallocated (pinned) array."""
    dt = NP_DTYPE[spec.dtype]
    g = rng(2, 0)
    if out is None:
        return g.random(spec.n, dtype=dt)
    g.random(spec.n, dtype=dt, out=out)
    return out


def partition_bounds(n: int, parts: int):
    """Contiguous partitions of n cells: the first n % parts get one extra cell."""
    base, extra = divmod(n, parts)
    bounds, off = [], 0
    for p in range(parts):
        size = base + (1 if p < extra else 0)
        bounds.append((off, size))
        off += size
    return bounds


def batched1d_problems(spec: Batched1D = Batched1D()):
    """(sizes int64[count], r float64[count], offsets int64[count]) — sizes
    floor(exp(U(ln nmin, ln nmax))) clamped to [nmin, nmax]."""
    g = rng(3, 0)
    sizes = np.floor(np.exp(g.uniform(math.log(spec.nmin), math.log(spec.nmax), spec.count)))
    sizes = np.clip(sizes, spec.nmin, spec.nmax).astype(np.int64)
    rs = rng(3, 1).uniform(spec.rmin, spec.rmax, spec.count)
    offsets = np.zeros(spec.count, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)[:-1]
    return sizes, rs, offsets


def batched1d_u0(spec: Batched1D = Batched1D(), total: int | None = None) -> np.ndarray:
    sizes, _, _ = batched1d_problems(spec)
    total = int(sizes.sum()) if total is None else total
    return rng(3, 2).random(total, dtype=NP_DTYPE[spec.dtype])


def gaussian_bumps(ny: int, nx: int, centres: int, sigma: float, workload_id: int,
                   dtype=np.float32) -> np.ndarray:
    """sum_c exp(-((i-yc)^2 + (j-xc)^2) / (2 sigma^2)), centres (yc, xc) ~
    U[0, ny) x U[0, nx); each bump is separable and truncated to |d| <= 8 sigma."""
    g = rng(workload_id, 10)
    yc = g.uniform(0, ny, centres)
    xc = g.uniform(0, nx, centres)
    u = np.zeros((ny, nx), dtype=np.float64)
    cut = int(math.ceil(8 * sigma))
    for c in range(centres):
        i0, i1 = max(0, int(math.floor(yc[c])) - cut), min(ny, int(math.ceil(yc[c])) + cut + 1)
        j0, j1 = max(0, int(math.floor(xc[c])) - cut), min(nx, int(math.ceil(xc[c])) + cut + 1)
        di = np.arange(i0, i1, dtype=np.float64) - yc[c]
        dj = np.arange(j0, j1, dtype=np.float64) - xc[c]
        gy = np.where(np.abs(di) <= 8 * sigma, np.exp(-di * di / (2 * sigma * sigma)), 0.0)
        gx = np.where(np.abs(dj) <= 8 * sigma, np.exp(-dj * dj / (2 * sigma * sigma)), 0.0)
        u[i0:i1, j0:j1] += np.outer(gy, gx)
    return u.astype(dtype)


def banded2d_u0(spec: Banded2D = Banded2D()) -> np.ndarray:
    return gaussian_bumps(spec.ny, spec.nx, spec.centres, spec.sigma, 4, NP_DTYPE[spec.dtype])


def band_bounds(ny: int, bands: int):
    return partition_bounds(ny, bands)


def varcoef2d_inputs(spec: VarCoef2D = VarCoef2D()):
    """(u0, kappa, target), each (ny, nx) of the run dtype."""
    dt = NP_DTYPE[spec.dtype]
    z = rng(5, 0).standard_normal((spec.ny, spec.nx))
    kappa = np.minimum(np.exp(spec.mu + spec.sigma_log * z), spec.kappa_max).astype(dt)
    u0 = gaussian_bumps(spec.ny, spec.nx, spec.centres, spec.sigma, 5, dt)
    target = rng(5, 1).random((spec.ny, spec.nx)).astype(dt)
    return u0, kappa, target


def uniform(shape, workload_id: int, stream: int, lo=0.0, hi=1.0, dtype=np.float64):
    """Generic seeded uniform array for small test cases."""
    return rng(workload_id, stream).uniform(lo, hi, shape).astype(dtype)
