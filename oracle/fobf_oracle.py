"""FP64 CPU oracle for "Optimized Fourier Bilateral Filtering" (Ghosh, Nair,
Chaudhury, IEEE Signal Processing Letters 25(10), 2018).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  The GPU
library never calls it, and it shares no code with the GPU library: it
depends on numpy (and scipy is used only by tests as an independent check).

Everything here is plain, slow and written to be compared with the paper by
eye, in float64:

* ``brute_bf``            eq. (1) with the Gaussian kernels of eq. (2),
                          by brute force over the square window of radius
                          ceil(3*theta) (the (6*theta+1)^2 window, Sec. I).
* ``fit_E`` / ``fit``     eq. (4)-(5): least-squares fit of the K cosine
                          coefficients of eq. (3) to the integer samples of
                          the range kernel, and the scan over the period T
                          of eq. (6) for fixed K.
* ``algorithm1``          Algorithm 1: smallest K with e(K) <= eps.
* ``lut_build`` /
  ``lut_fit``             the offline (sigma, eps) -> (K*, T*) table and its
                          bilinear read-out (Sec. II, after Algorithm 1).
* ``fourier_direct``      the K-term shiftable filter (eq. (1) with the
                          cosine series of eq. (3) as range kernel, written
                          as spatial convolutions, Sec. II first paragraph),
                          by direct separable convolution of the channels.
* ``brute_bf_points``     eq. (1) at selected pixels, any range kernel.
* ``psnr`` / ``max_abs``  the accuracy metric of Sec. III.

Readings of points the paper leaves open:

1. Period: frequencies are 2*pi*k/(2T+1) exactly as eq. (3) writes them.
2. Window: square, radius r = ceil(3*theta); unnormalised taps,
   omega(0) = 1 (normalisation cancels in every ratio of eq. (1)).
3. Image boundary: neighbours outside the image are left out of both sums
   of eq. (1).  In the convolution form this is zero padding of every
   channel, including the constant channel, whose blur W(i) is therefore
   not constant near the border.
4. Ties in the T scan: the smallest T among exactly equal errors.
5. The filter output is N/D literally (no clamp); D can be <= 0 where the
   cosine series goes negative.
6. Table read-out: bilinear in (sigma, log(1/eps)); the interpolated order
   is rounded up and the period to the nearest integer (at least K - 1).
"""
from __future__ import annotations

import math

import numpy as np

# --------------------------------------------------------------------------
# Kernels, eq. (2)
# --------------------------------------------------------------------------


def spatial_radius(theta: float) -> int:
    """Radius of the square spatial window: ceil(3*theta) (Sec. I)."""
    if not (theta > 0.0 and math.isfinite(theta)):
        raise ValueError("theta must be positive and finite")
    return int(math.ceil(3.0 * theta))


def spatial_taps(theta: float) -> np.ndarray:
    """1-D taps g(m) = exp(-m^2 / (2 theta^2)), m = -r..r (eq. (2)).

    The 2-D spatial kernel is omega(jy, jx) = g(jy) * g(jx)."""
    r = spatial_radius(theta)
    m = np.arange(-r, r + 1, dtype=np.float64)
    return np.exp(-(m * m) / (2.0 * theta * theta))


def gaussian_range(sigma: float):
    """Range kernel phi(t) = exp(-t^2 / (2 sigma^2)) of eq. (2)."""
    s2 = 2.0 * float(sigma) * float(sigma)

    def phi(t):
        t = np.asarray(t, dtype=np.float64)
        return np.exp(-(t * t) / s2)

    return phi


def cosine_series(c, T: int):
    """phi_hat(t) = sum_{k<K} c_k cos(2 pi k t / (2T+1)), eq. (3)."""
    c = np.asarray(c, dtype=np.float64)
    nu = 2.0 * math.pi / (2 * T + 1)

    def phi_hat(t):
        t = np.asarray(t, dtype=np.float64)
        out = np.zeros_like(t)
        for k in range(len(c)):
            out = out + c[k] * np.cos(nu * k * t)
        return out

    return phi_hat


# --------------------------------------------------------------------------
# Brute force, eq. (1)
# --------------------------------------------------------------------------


def brute_bf(f: np.ndarray, theta: float, range_kernel, return_nd=False):
    """Bilateral filter eq. (1) by brute force.

    For each pixel i, sums over offsets j in the square window of radius
    r = ceil(3 theta): omega(j) * phi(f(i-j) - f(i)) * f(i-j) (numerator) and
    omega(j) * phi(f(i-j) - f(i)) (denominator), keeping only neighbours
    i-j that lie inside the image.  Vectorised over pixels, looping over j.
    """
    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape
    r = spatial_radius(theta)
    g = spatial_taps(theta)
    num = np.zeros((H, W))
    den = np.zeros((H, W))
    for jy in range(-r, r + 1):
        for jx in range(-r, r + 1):
            w = g[jy + r] * g[jx + r]
            if abs(jy) >= H or abs(jx) >= W:
                continue          # no pixel has this neighbour in the image
            # neighbour i - j for every pixel i; valid where inside image
            nb = np.zeros((H, W))
            valid = np.zeros((H, W), dtype=bool)
            ys = slice(max(0, jy), min(H, H + jy))
            xs = slice(max(0, jx), min(W, W + jx))
            ys_n = slice(max(0, jy) - jy, min(H, H + jy) - jy)
            xs_n = slice(max(0, jx) - jx, min(W, W + jx) - jx)
            nb[ys, xs] = f[ys_n, xs_n]
            valid[ys, xs] = True
            wt = np.where(valid, w * range_kernel(nb - f), 0.0)
            num += wt * nb
            den += wt
    out = num / den
    if return_nd:
        return out, num, den
    return out


def brute_bf_points(f: np.ndarray, theta: float, range_kernel, ys, xs):
    """eq. (1) evaluated only at pixels (ys[n], xs[n]); same rules as
    :func:`brute_bf`.  Used to check very large images at sampled pixels.
    Returns (out, num, den) as 1-D arrays."""
    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape
    r = spatial_radius(theta)
    g = spatial_taps(theta)
    ys = np.asarray(ys, dtype=np.int64)
    xs = np.asarray(xs, dtype=np.int64)
    out = np.empty(len(ys))
    num = np.empty(len(ys))
    den = np.empty(len(ys))
    for n in range(len(ys)):
        y, x = int(ys[n]), int(xs[n])
        y0, y1 = max(0, y - r), min(H, y + r + 1)
        x0, x1 = max(0, x - r), min(W, x + r + 1)
        win = f[y0:y1, x0:x1]
        w = np.outer(g[y0 - y + r:y1 - y + r], g[x0 - x + r:x1 - x + r])
        wt = w * range_kernel(win - f[y, x])
        num[n] = np.sum(wt * win)
        den[n] = np.sum(wt)
        out[n] = num[n] / den[n]
    return out, num, den


# --------------------------------------------------------------------------
# Least-squares fit, eq. (4)-(6), Algorithm 1
# --------------------------------------------------------------------------


def design_matrix(R: int, K: int, T: int):
    """A (2R+1 x K) with A[i, j] = cos(nu * t_i * j), t_i = i - R (0-based
    i), nu = 2 pi / (2T+1), as defined below eq. (4)."""
    t = np.arange(-R, R + 1, dtype=np.float64)
    nu = 2.0 * math.pi / (2 * T + 1)
    k = np.arange(K, dtype=np.float64)
    return np.cos(nu * np.outer(t, k)), t


def fit_E(R: int, sigma_or_samples, K: int, T: int):
    """Coefficients c minimising ||A c - b||^2 and the minimum E(K, T),
    eq. (5).  ``sigma_or_samples`` is sigma (Gaussian range kernel, b(t) =
    phi(t)) or a callable giving the target kernel's samples b(t).

    Solved with numpy's SVD least squares (minimum-norm c when A is rank
    deficient); E is computed from the residual A c - b itself."""
    A, t = design_matrix(R, K, T)
    if callable(sigma_or_samples):
        b = np.asarray(sigma_or_samples(t), dtype=np.float64)
    else:
        b = gaussian_range(sigma_or_samples)(t)
    c, *_ = np.linalg.lstsq(A, b, rcond=None)
    res = A @ c - b
    return c, float(np.dot(res, res))


def fit(R: int, sigma_or_samples, K: int, Tmax: int | None = None):
    """Fixed-order fit: T* = argmin_{1 <= T <= Tmax} E(K, T) (eq. (6) with
    the search range of Algorithm 1), smallest T on exact ties.

    Returns dict(T, c, E, delta, Es) where delta = max_t |phi - phi_hat| on
    the integers -R..R and Es[T-1] = E(K, T)."""
    if Tmax is None:
        Tmax = 4 * R
    Es = np.empty(Tmax)
    cs = []
    for T in range(1, Tmax + 1):
        c, E = fit_E(R, sigma_or_samples, K, T)
        Es[T - 1] = E
        cs.append(c)
    i = int(np.argmin(Es))          # first index of the minimum
    T = i + 1
    c = cs[i]
    return {"T": T, "c": c, "E": float(Es[i]),
            "delta": kernel_maxdev(R, sigma_or_samples, c, T), "Es": Es}


def kernel_maxdev(R, sigma_or_samples, c, T):
    """max over integers t in [-R, R] of |phi(t) - phi_hat(t)|."""
    t = np.arange(-R, R + 1, dtype=np.float64)
    if callable(sigma_or_samples):
        b = np.asarray(sigma_or_samples(t), dtype=np.float64)
    else:
        b = gaussian_range(sigma_or_samples)(t)
    return float(np.max(np.abs(cosine_series(c, T)(t) - b)))


def algorithm1(R: int, sigma_or_samples, eps: float, Tmax: int | None = None,
               Kmax: int = 64):
    """Algorithm 1: raise K from 1 until the best error over the period scan
    is within eps.  For each K the scan over T = 1..Tmax keeps the T with
    the smallest E(K, T) among those <= eps (first such T on exact ties).
    Returns dict(K, T, c, E)."""
    if Tmax is None:
        Tmax = 4 * R
    e = math.inf
    best = None
    K = 0
    while e > eps:
        K += 1
        if K > Kmax:
            raise RuntimeError("no order up to Kmax meets eps")
        for T in range(1, Tmax + 1):
            c, e0 = fit_E(R, sigma_or_samples, K, T)
            if e0 <= eps and e0 < e:
                best = {"K": K, "T": T, "c": c, "E": e0}
                e = e0
    return best


def lut_build(R: int, sigmas, eps_list, Tmax: int | None = None):
    """The offline table of Sec. II (paragraph after Algorithm 1, Fig. 2):
    (K*, T*) of Algorithm 1 at every (sigma, eps) grid point.  Returns
    dict(sigmas, eps, K[i][j], T[i][j])."""
    K = [[0] * len(eps_list) for _ in sigmas]
    T = [[0] * len(eps_list) for _ in sigmas]
    for i, s in enumerate(sigmas):
        for j, e in enumerate(eps_list):
            r = algorithm1(R, float(s), float(e), Tmax)
            K[i][j], T[i][j] = r["K"], r["T"]
    return {"R": R, "sigmas": [float(x) for x in sigmas],
            "eps": [float(x) for x in eps_list], "K": K, "T": T}


def lut_interp(table, sigma: float, eps: float):
    """Bilinear read-out of the table at an off-grid (sigma, eps), in the
    coordinates (sigma, log(1/eps)) in which the paper reports K* and T*
    varying smoothly and almost linearly.  The order is rounded up, the
    period to the nearest integer (and kept >= K - 1).  Returns (K, T)."""
    sg = table["sigmas"]
    L = [-math.log(e) for e in table["eps"]]
    x, y = float(sigma), -math.log(eps)

    def cell(g, v):
        if len(g) == 1:
            if v != g[0]:
                raise ValueError("outside the table")
            return 0, 0, 0.0
        if not (g[0] <= v <= g[-1]):
            raise ValueError("outside the table")
        i = 0
        while i < len(g) - 2 and v >= g[i + 1]:
            i += 1
        return i, i + 1, (v - g[i]) / (g[i + 1] - g[i])

    i0, i1, a = cell(sg, x)
    j0, j1, b = cell(L, y)

    def bil(M):
        return ((1 - a) * ((1 - b) * M[i0][j0] + b * M[i0][j1])
                + a * ((1 - b) * M[i1][j0] + b * M[i1][j1]))

    K = int(math.ceil(bil(table["K"]) - 1e-9))
    T = max(max(1, K - 1), int(math.floor(bil(table["T"]) + 0.5)))
    return K, T


def lut_fit(table, sigma: float, eps: float):
    """Run-time step of the table: (K, T) by :func:`lut_interp`, then the
    least-squares coefficients at that (K, T), eq. (5).  Returns dict(K, T,
    c, E)."""
    K, T = lut_interp(table, sigma, eps)
    c, E = fit_E(table["R"], float(sigma), K, T)
    return {"K": K, "T": T, "c": c, "E": E}


# --------------------------------------------------------------------------
# The K-term shiftable (Fourier) filter by direct convolution
# --------------------------------------------------------------------------


def conv_zero(X: np.ndarray, g: np.ndarray) -> np.ndarray:
    """(omega * X)(i) = sum_j omega(j) X(i-j) over in-image neighbours only
    (zero padding), omega = g (x) g; rows first, then columns."""
    H, W = X.shape
    r = (len(g) - 1) // 2
    tmp = np.zeros((H, W))
    for m in range(-r, r + 1):
        # tmp(y, x) += g(m) * X(y, x - m), x - m inside [0, W)
        lo, hi = max(0, m), min(W, W + m)
        if lo < hi:
            tmp[:, lo:hi] += g[m + r] * X[:, lo - m:hi - m]
    out = np.zeros((H, W))
    for m in range(-r, r + 1):
        lo, hi = max(0, m), min(H, H + m)
        if lo < hi:
            out[lo:hi, :] += g[m + r] * tmp[lo - m:hi - m, :]
    return out


def fourier_direct(f: np.ndarray, theta: float, K: int, T: int, c,
                   return_nd=False):
    """Fourier bilateral filter: eq. (1) with phi replaced by the cosine
    series phi_hat of eq. (3), computed through spatial convolutions.

    With nu = 2 pi / (2T+1), C_k = cos(nu k f), S_k = sin(nu k f) and the
    angle-difference identity cos(nu k (f(i-j) - f(i))) =
    C_k(i-j) C_k(i) + S_k(i-j) S_k(i):

      N(i) = c_0 (w*f)(i) + sum_{k>=1} c_k [C_k(i) (w*(C_k f))(i)
                                            + S_k(i) (w*(S_k f))(i)]
      D(i) = c_0 (w*1)(i) + sum_{k>=1} c_k [C_k(i) (w*C_k)(i)
                                            + S_k(i) (w*S_k)(i)]

    output N / D.  Convolutions are zero padded (neighbours outside the
    image do not count), matching :func:`brute_bf`."""
    f = np.asarray(f, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    if len(c) != K:
        raise ValueError("len(c) must equal K")
    g = spatial_taps(theta)
    nu = 2.0 * math.pi / (2 * T + 1)
    num = c[0] * conv_zero(f, g)
    den = c[0] * conv_zero(np.ones_like(f), g)
    for k in range(1, K):
        C = np.cos(nu * k * f)
        S = np.sin(nu * k * f)
        num += c[k] * (C * conv_zero(C * f, g) + S * conv_zero(S * f, g))
        den += c[k] * (C * conv_zero(C, g) + S * conv_zero(S, g))
    out = num / den
    if return_nd:
        return out, num, den
    return out


def blur_weight(H: int, W: int, theta: float) -> np.ndarray:
    """W(i) = sum of omega(j) over in-image neighbours (the blur of the
    constant image)."""
    return conv_zero(np.ones((H, W)), spatial_taps(theta))


# --------------------------------------------------------------------------
# Metrics (Sec. III)
# --------------------------------------------------------------------------


def psnr(ref: np.ndarray, test: np.ndarray, peak: float = 255.0) -> float:
    """PSNR = 10 log10(255^2 / MSE)."""
    d = np.asarray(ref, dtype=np.float64) - np.asarray(test, dtype=np.float64)
    mse = float(np.mean(d * d))
    if mse == 0.0:
        return math.inf
    return 10.0 * math.log10(peak * peak / mse)


def max_abs(ref: np.ndarray, test: np.ndarray, mask=None) -> float:
    d = np.abs(np.asarray(ref, dtype=np.float64)
               - np.asarray(test, dtype=np.float64))
    if mask is not None:
        d = d[mask]
    return float(np.max(d)) if d.size else 0.0


def prop1_bound(R: int, delta: float, Wi: np.ndarray) -> np.ndarray:
    """Per-pixel bound on |Fourier filter - brute force| for images with
    values in [0, R]: R delta W(i) / (omega(0) - delta W(i)), omega(0) = 1,
    where delta bounds |phi - phi_hat| on the integers of [-R, R]
    (Proposition 1 restated with a max-norm kernel error and unnormalised
    omega; +inf where delta W(i) >= 1)."""
    dw = delta * np.asarray(Wi, dtype=np.float64)
    with np.errstate(divide="ignore"):
        return np.where(dw < 1.0, R * dw / (1.0 - dw), np.inf)
