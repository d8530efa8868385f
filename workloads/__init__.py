"""Seeded synthetic workloads for the Fourier bilateral filter.

This module only draws random numbers and lays out images and request
streams.  It holds none of the filter's arithmetic, so both the FP64 oracle
(``oracle/``) and the GPU path may import it without sharing any method code.

The paper measures on 8-bit grayscale photographs (Sec. III: BM3D images,
R = 255).  Those images are not available, so the generator below stands in
for them: piecewise-constant Voronoi cells with sharp edges (what the range
kernel must preserve), an optional smooth sinusoidal ramp, Gaussian noise,
clipped and rounded to integers in [0, 255] like 8-bit data.

Workloads
---------
C1  256x256, 16 cells, no ramp, seed 1001; theta=3, sigma=30, K=4, eps=0.1.
C2  1024x1024, 64 cells, ramp, seed 1002; theta=5, sigma in {10,30,80}, K=6.
C3  4096x4096, 256 cells, ramp, seed 1003; theta=10, sigma in {20,50,100}, K=8.
C4  256 images of uneven size/params (seed 1004+i), see :func:`batch_jobs`.
C5  Poisson request stream (seed 1005), see :func:`serve_stream`.
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass

import numpy as np

R_DEFAULT = 255


def _rng(seed):
    if isinstance(seed, np.random.Generator):
        return seed
    return np.random.default_rng(seed)


def voronoi_image(H: int, W: int, ncells: int, ramp: bool, seed) -> np.ndarray:
    """Voronoi + ramp + noise image, float64, integer-valued in [0, 255].

    Draw order (numpy PCG64): seed rows, seed cols, cell values, noise.
    Labels go to the nearest seed (Euclidean) of each integer pixel centre;
    seeds are continuous uniform, so exact distance ties have probability 0.
    """
    from scipy.spatial import cKDTree

    rng = _rng(seed)
    sy = rng.uniform(0.0, H, ncells)
    sx = rng.uniform(0.0, W, ncells)
    v = rng.uniform(0.0, 255.0, ncells)
    tree = cKDTree(np.stack([sy, sx], axis=1))
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64),
                         np.arange(W, dtype=np.float64), indexing="ij")
    _, label = tree.query(np.stack([yy.ravel(), xx.ravel()], axis=1), k=1,
                          workers=-1)
    f = v[label].reshape(H, W)
    if ramp:
        f = f + 32.0 * np.sin(2.0 * math.pi * (1.5 * xx / W + 0.75 * yy / H))
    f = f + rng.normal(0.0, 10.0, size=(H, W))
    return np.rint(np.clip(f, 0.0, 255.0))


@functools.lru_cache(maxsize=4)
def _cached_image(H, W, ncells, ramp, seed):
    img = voronoi_image(H, W, ncells, ramp, seed)
    img.setflags(write=False)
    return img


def image(H, W, ncells, ramp, seed) -> np.ndarray:
    """Cached read-only copy of :func:`voronoi_image` (integer seeds only)."""
    return _cached_image(int(H), int(W), int(ncells), bool(ramp), int(seed))


@dataclass(frozen=True)
class Config:
    name: str
    H: int
    W: int
    ncells: int
    ramp: bool
    seed: int
    theta: float
    sigmas: tuple
    K: int
    R: int = R_DEFAULT
    eps: float = 0.1

    def image(self) -> np.ndarray:
        return image(self.H, self.W, self.ncells, self.ramp, self.seed)


C1 = Config("C1", 256, 256, 16, False, 1001, 3.0, (30.0,), 4)
C2 = Config("C2", 1024, 1024, 64, True, 1002, 5.0, (10.0, 30.0, 80.0), 6)
C3 = Config("C3", 4096, 4096, 256, True, 1003, 10.0, (20.0, 50.0, 100.0), 8)


@dataclass(frozen=True)
class Job:
    """One image of the uneven batch (C4) or one serving request (C5)."""
    H: int
    W: int
    ncells: int
    theta: float
    sigma: float
    K: int
    seed: int
    prec: int = 0          # 0 = fp32, 1 = fp16-staged, 2 = bf16-staged
    t_arrival: float = 0.0


def batch_jobs(n: int = 256, base_seed: int = 1004, area_lo: int = 64 * 64,
               area_hi: int = 2048 * 2048) -> list:
    """C4: n images, log-uniform area, log-uniform aspect in [1/4, 4].

    Per image i (generator seeded 1004+i): area, aspect, theta ~ U[2,8],
    sigma = round(U[10,80]), K ~ U{3..10}; the image itself is drawn from
    the same generator afterwards (see :func:`job_image`).
    """
    jobs = []
    for i in range(n):
        rng = np.random.default_rng(base_seed + i)
        A = math.exp(rng.uniform(math.log(area_lo), math.log(area_hi)))
        a = math.exp(rng.uniform(math.log(0.25), math.log(4.0)))
        H = max(8, int(round(math.sqrt(A * a))))
        W = max(8, int(round(A / H)))
        ncells = max(4, int(round(math.sqrt(H * W) / 16.0)))
        theta = float(rng.uniform(2.0, 8.0))
        sigma = float(round(rng.uniform(10.0, 80.0)))
        K = int(rng.integers(3, 11))
        jobs.append(Job(H, W, ncells, theta, sigma, K, base_seed + i))
    return jobs


def job_image(job: Job) -> np.ndarray:
    """Image of a batch job: Voronoi+ramp+noise from seed (job.seed, 7)."""
    return voronoi_image(job.H, job.W, job.ncells, True,
                         np.random.default_rng([job.seed, 7]))


def serve_stream(n: int = 4400, rate: float = 200.0, seed: int = 1005,
                 side_lo: int = 128, side_hi: int = 4096,
                 thetas=(2.0, 10.0), sigmas=(10.0, 100.0),
                 Ks=(4, 6, 8)) -> list:
    """C5: Poisson arrivals (exponential gaps, mean 1/rate seconds).

    Square images with log-uniform area (so log-uniform side), theta ~
    U[thetas], sigma = round(U[sigmas]), K uniform over Ks; even request
    index -> fp32, odd -> fp16-staged.  Image content comes from
    :func:`request_image` (crops of one pool image), not from this list.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += float(rng.exponential(1.0 / rate))
        side = int(round(math.exp(rng.uniform(math.log(side_lo),
                                              math.log(side_hi)))))
        theta = float(rng.uniform(*thetas))
        sigma = float(round(rng.uniform(*sigmas)))
        K = int(Ks[int(rng.integers(0, len(Ks)))])
        out.append(Job(side, side, 0, theta, sigma, K, seed, i % 2, t))
    return out


def request_image(pool: np.ndarray, job: Job, index: int) -> np.ndarray:
    """Crop of a pool image for serving request ``index`` (deterministic)."""
    PH, PW = pool.shape
    h, w = min(job.H, PH), min(job.W, PW)
    rng = np.random.default_rng([job.seed, index])
    y = int(rng.integers(0, PH - h + 1))
    x = int(rng.integers(0, PW - w + 1))
    return pool[y:y + h, x:x + w]
