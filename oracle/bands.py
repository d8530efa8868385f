"""Whole-image oracle over row bands in worker processes.

TEST INFRASTRUCTURE ONLY (same rule as fobf_oracle.py: only ``tests/``,
``__graft_entry__.smoke()`` and the oracle legs of ``bench.py`` use it).

``fourier_direct`` of the oracle evaluated on the rows [a, b) of an image,
where a = max(0, y0 - r) and b = min(H, y1 + r), gives rows [y0, y1) of the
whole-image result exactly, bit for bit: every output row's horizontal pass
and its pointwise products depend on that row only, and the vertical sum of
a kept row reaches rows inside [a, b) (or outside the image, excluded in
both cases) in the same order of taps.  The band boundaries are therefore
invisible in the result; the same holds for the in-image tap sum W(i)
(``blur_weight``).  This module only splits the image and stacks the
bands; all arithmetic is fobf_oracle's.

Workers are started with the "spawn" method, so a parent that has already
opened a GPU context forks nothing of it; they import numpy and the oracle
only.
"""
from __future__ import annotations

import math
import multiprocessing as mp
import os

import numpy as np

from . import fobf_oracle as O


def _band_job(args):
    band, theta, K, T, c, top, rows = args
    out, num, den = O.fourier_direct(band, theta, K, T, c, return_nd=True)
    Wi = O.blur_weight(band.shape[0], band.shape[1], theta)
    sl = slice(top, top + rows)
    return out[sl], num[sl], den[sl], Wi[sl]


def band_jobs(f, theta, K, T, c, nbands):
    """Argument tuples of the bands: each band holds its kept rows plus up to
    r = ceil(3 theta) halo rows above and below."""
    f = np.asarray(f, dtype=np.float64)
    H = f.shape[0]
    r = O.spatial_radius(theta)
    step = max(1, (H + nbands - 1) // nbands)
    jobs = []
    for y0 in range(0, H, step):
        y1 = min(H, y0 + step)
        a, b = max(0, y0 - r), min(H, y1 + r)
        jobs.append((np.ascontiguousarray(f[a:b]), float(theta), int(K), int(T),
                     np.asarray(c, dtype=np.float64), y0 - a, y1 - y0))
    return jobs


def default_workers() -> int:
    """Worker processes: the host's cores, at most 16."""
    return max(1, min(16, os.cpu_count() or 1))


class BandPool:
    """A pool of spawned workers that runs the oracle's Fourier filter over
    row bands.  Use as a context manager; ``fourier_direct`` returns
    (out, num, den, W) of the whole image, equal bit for bit to the
    single-process oracle (and ``blur_weight``)."""

    def __init__(self, workers: int | None = None):
        self.workers = workers or default_workers()
        self._pool = mp.get_context("spawn").Pool(self.workers)

    def fourier_direct(self, f, theta, K, T, c, nbands: int | None = None):
        jobs = band_jobs(f, theta, K, T, c, nbands or 2 * self.workers)
        parts = self._pool.map(_band_job, jobs)
        return tuple(np.concatenate([p[i] for p in parts], axis=0) for i in range(4))

    def close(self):
        if self._pool is not None:
            self._pool.close()
            self._pool.join()
            self._pool = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def full_image_stats(got, ref, den, Wi, dmask: float = 0.01):
    """Accuracy of an output against the oracle on every pixel (Sec. III's
    metrics): pixels whose oracle denominator satisfies D/W < dmask are
    masked (counted, and their error reported separately); PSNR is over the
    whole image and over the unmasked pixels."""
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - ref)
    mask = (den / Wi) >= dmask
    n_masked = int(mask.size - np.count_nonzero(mask))
    finite = np.isfinite(err)
    e_un = float(err[mask].max()) if mask.any() else 0.0
    e_all = float(err.max()) if finite.all() else math.inf
    e_m = float(err[~mask].max()) if n_masked and np.isfinite(err[~mask]).all() else (
        0.0 if not n_masked else math.inf)

    def psnr(sel):
        d = err[sel] if sel is not None else err
        if d.size == 0 or not np.isfinite(d).all():
            return None
        mse = float(np.mean(d * d))
        return math.inf if mse == 0.0 else 10.0 * math.log10(255.0 ** 2 / mse)

    return {"pixels": int(err.size), "masked": n_masked, "maxabs_unmasked": e_un,
            "maxabs_masked": e_m, "maxabs_all": e_all, "psnr_all_db": psnr(None),
            "psnr_unmasked_db": psnr(mask), "min_dw": float(np.min(den / Wi))}
