"""Pins for the FP64 oracle: each test ties it to something other than
itself (a value the paper prints, a closed form, a library routine in a
special case, an exact identity, or an invariant)."""
import json
import math
import os

import numpy as np
import pytest
from scipy import ndimage

import oracle as O
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_image(H=23, W=31, seed=5, ncells=6):
    return workloads.voronoi_image(H, W, ncells, True, seed)


# ------------------------------------------------------------------ fit ---

def test_fig1_worked_example():
    """Sec. II, Fig. 1: E(4, T) is minimised at T = 203 (R=255, sigma=50);
    T = 150 and T = 350 are poor, i.e. above the tolerance 0.1."""
    g = json.load(open(os.path.join(GOLDEN, "fig1_worked_example.json")))
    r = O.fit(g["R"], g["sigma"], g["K"])
    assert r["T"] == g["T_star"]
    assert r["E"] <= g["eps"]
    for T in g["T_poor"]:
        _, E = O.fit_E(g["R"], g["sigma"], g["K"], T)
        assert E > g["eps"]


def test_algorithm1_fig1_setting():
    """Algorithm 1 at sigma=50, eps=0.1 stops at K=4 (the order Fig. 1 uses
    with that tolerance) with T* = 203, and e(3) > eps >= e(4)."""
    g = json.load(open(os.path.join(GOLDEN, "fig1_worked_example.json")))
    a = O.algorithm1(g["R"], g["sigma"], g["eps"])
    assert a["K"] == 4 and a["T"] == 203
    assert O.fit(255, 50.0, 3)["E"] > 0.1


def test_closed_form_at_T_equal_R():
    """With T = R the K columns are orthogonal over the 2R+1 integers of
    [-R, R] (discrete Fourier orthogonality), so the least-squares
    coefficients are the DFT coefficients: c_0 = mean(phi), c_k =
    2/(2R+1) sum_t phi(t) cos(2 pi k t / (2R+1))."""
    for R, sigma, K in [(255, 50.0, 6), (255, 20.0, 8), (31, 7.0, 5)]:
        t = np.arange(-R, R + 1)
        phi = np.exp(-t * t / (2 * sigma * sigma))
        n = 2 * R + 1
        ck = [phi.sum() / n] + [
            2.0 / n * np.sum(phi * np.cos(2 * math.pi * k * t / n))
            for k in range(1, K)]
        c, E = O.fit_E(R, sigma, K, R)
        np.testing.assert_allclose(c, ck, rtol=0, atol=1e-14)
        # Parseval: E = ||phi||^2 - n c_0^2 - n/2 sum_k c_k^2
        parseval = (np.sum(phi * phi) - n * ck[0] ** 2
                    - n / 2 * sum(x * x for x in ck[1:]))
        assert E == pytest.approx(parseval, rel=1e-9, abs=1e-12)


def test_exact_interpolation_prop2():
    """Proposition 2: the error vanishes once the order reaches 2R+1; with
    T = R already K = R+1 cosines interpolate every even function on the
    2R+1 integers."""
    c, E = O.fit_E(255, 50.0, 256, 255)
    assert E < 1e-24
    R = 6
    assert O.fit(R, 3.0, 2 * R + 1, Tmax=40)["E"] < 1e-26


def test_monotone_in_K():
    """Proposition 2: e(K+1) <= e(K); also E(K+1,T) <= E(K,T) for each T
    (nested column spaces)."""
    prev = math.inf
    for K in range(1, 8):
        e = O.fit(255, 30.0, K, Tmax=600)["E"]
        assert e <= prev * (1 + 1e-9) + 1e-15
        prev = e
    for T in (40, 160, 400):
        Es = [O.fit_E(255, 30.0, K, T)[1] for K in range(1, 9)]
        assert all(b <= a * (1 + 1e-9) + 1e-15 for a, b in zip(Es, Es[1:]))


def test_flat_kernel_degenerate():
    """sigma -> infinity: b = 1 is fitted exactly by c = (1, 0, ..., 0) for
    every T; the scan returns the smallest T."""
    r = O.fit(255, lambda t: np.ones_like(t), 4, Tmax=50)
    assert r["E"] < 1e-25
    np.testing.assert_allclose(r["c"], [1, 0, 0, 0], atol=1e-12)
    assert r["T"] == 1 or r["Es"][r["T"] - 1] <= r["Es"].min()


def test_fit_nongaussian_kernel():
    """The fit takes arbitrary samples b(t) (Sec. I, contributions): a kernel
    that is itself a cosine series of period 2T+1 is recovered exactly."""
    T = 90
    c_true = np.array([0.3, 0.5, -0.2])
    phi = O.cosine_series(c_true, T)
    c, E = O.fit_E(255, phi, 3, T)
    np.testing.assert_allclose(c, c_true, atol=1e-12)
    assert E < 1e-24


# --------------------------------------------------------- brute force ---

def test_brute_bf_flat_range_is_gaussian_blur():
    """phi == 1 turns eq. (1) into a normalised Gaussian blur (zero
    outside the image): scipy.ndimage.correlate with mode='constant'."""
    f = small_image()
    theta = 1.7
    g = O.spatial_taps(theta)
    w2 = np.outer(g, g)
    ref = (ndimage.correlate(f, w2, mode="constant")
           / ndimage.correlate(np.ones_like(f), w2, mode="constant"))
    out = O.brute_bf(f, theta, lambda t: np.ones_like(t))
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-10)


def test_brute_bf_two_level_image():
    """Image with two levels a, b: at a pixel of level a, eq. (1) gives
    (a Wa + b phi(b-a) Wb) / (Wa + phi(b-a) Wb), with Wa, Wb the spatial
    weight of each level's pixels in the window (linear filtering of the
    indicator images by scipy)."""
    rng = np.random.default_rng(3)
    H, W = 19, 26
    a, b = 40.0, 90.0
    mask = rng.random((H, W)) < 0.4
    f = np.where(mask, b, a)
    theta, sigma = 1.3, 35.0
    g = O.spatial_taps(theta)
    w2 = np.outer(g, g)
    Wa = ndimage.correlate((~mask).astype(float), w2, mode="constant")
    Wb = ndimage.correlate(mask.astype(float), w2, mode="constant")
    p = math.exp(-(b - a) ** 2 / (2 * sigma * sigma))
    ref = np.where(mask, (b * Wb + a * p * Wa) / (Wb + p * Wa),
                   (a * Wa + b * p * Wb) / (Wa + p * Wb))
    out = O.brute_bf(f, theta, O.gaussian_range(sigma))
    np.testing.assert_allclose(out, ref, rtol=1e-12)


def test_brute_bf_invariants():
    f = small_image()
    theta, sigma = 1.5, 20.0
    phi = O.gaussian_range(sigma)
    out = O.brute_bf(f, theta, phi)
    # convex combination of window values
    r = O.spatial_radius(theta)
    lo = ndimage.minimum_filter(f, size=2 * r + 1, mode="nearest")
    hi = ndimage.maximum_filter(f, size=2 * r + 1, mode="nearest")
    assert np.all(out >= lo - 1e-9) and np.all(out <= hi + 1e-9)
    np.testing.assert_allclose(O.brute_bf(f.T, theta, phi), out.T, atol=1e-10)
    np.testing.assert_allclose(O.brute_bf(f[::-1, ::-1], theta, phi),
                               out[::-1, ::-1], atol=1e-10)
    np.testing.assert_allclose(O.brute_bf(f + 7.0, theta, phi), out + 7.0,
                               atol=1e-10)
    np.testing.assert_allclose(O.brute_bf(255.0 - f, theta, phi), 255.0 - out,
                               atol=1e-10)
    const = np.full((9, 13), 77.0)
    np.testing.assert_allclose(O.brute_bf(const, theta, phi), const,
                               atol=1e-12)
    # sigma -> 0 on an integer image: only equal neighbours count
    delta = lambda t: (np.abs(t) < 0.5).astype(float)  # noqa: E731
    np.testing.assert_allclose(O.brute_bf(f, theta, delta), f, atol=1e-12)


def test_brute_bf_matches_four_nested_loops():
    """eq. (1) written as the plainest possible loops (pixel, then every
    in-image neighbour of the square window) on a tiny image, with an
    asymmetric range kernel so that a swapped difference would show."""
    f = small_image(H=9, W=11, seed=3, ncells=4)
    theta = 1.2
    r = O.spatial_radius(theta)
    kernel = lambda t: np.exp(-(np.asarray(t) - 3.0) ** 2 / 800.0)  # noqa: E731
    H, W = f.shape
    ref = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            num = den = 0.0
            for jy in range(-r, r + 1):
                for jx in range(-r, r + 1):
                    yy, xx = y - jy, x - jx
                    if 0 <= yy < H and 0 <= xx < W:
                        w = math.exp(-(jy * jy + jx * jx) / (2 * theta * theta))
                        wt = w * float(kernel(f[yy, xx] - f[y, x]))
                        num += wt * f[yy, xx]
                        den += wt
            ref[y, x] = num / den
    np.testing.assert_allclose(O.brute_bf(f, theta, kernel), ref, rtol=1e-13, atol=1e-12)


def test_brute_bf_points_matches_full():
    f = small_image()
    theta = 2.2
    phi = O.gaussian_range(25.0)
    full = O.brute_bf(f, theta, phi)
    ys = np.array([0, 0, 22, 11, 5, 22])
    xs = np.array([0, 30, 30, 15, 0, 7])
    pts, _, _ = O.brute_bf_points(f, theta, phi, ys, xs)
    np.testing.assert_allclose(pts, full[ys, xs], rtol=1e-13)


# ----------------------------------------------------- Fourier filter ---

def test_conv_zero_matches_scipy():
    """Separable zero-padded convolution of a non-square array equals
    scipy.ndimage.correlate with the outer-product kernel."""
    rng = np.random.default_rng(2)
    X = rng.normal(size=(17, 29))
    g = O.spatial_taps(2.1)
    ref = ndimage.correlate(X, np.outer(g, g), mode="constant")
    np.testing.assert_allclose(O.conv_zero(X, g), ref, rtol=1e-12,
                               atol=1e-12)
    # radius larger than the image itself
    Y = rng.normal(size=(4, 3))
    ref = ndimage.correlate(Y, np.outer(g, g), mode="constant")
    np.testing.assert_allclose(O.conv_zero(Y, g), ref, atol=1e-12)


@pytest.mark.parametrize("K,T,theta", [(4, 161, 1.0), (6, 141, 1.7),
                                       (3, 5, 2.4), (8, 408, 1.2)])
def test_fourier_equals_bruteforce_with_series_kernel(K, T, theta):
    """The shiftable expansion is exact: the convolution form equals eq. (1)
    with phi_hat as range kernel, for any coefficients (random here,
    including ones that make D change sign)."""
    f = small_image()
    rng = np.random.default_rng(K * 1000 + T)
    c = rng.normal(size=K)
    c[0] += 1.0
    out, num, den = O.fourier_direct(f, theta, K, T, c, return_nd=True)
    ref, rnum, rden = O.brute_bf(f, theta, O.cosine_series(c, T),
                                 return_nd=True)
    scale = np.max(np.abs(rden))
    np.testing.assert_allclose(num, rnum, atol=1e-10 * scale * 255)
    np.testing.assert_allclose(den, rden, atol=1e-10 * scale)
    ok = np.abs(rden) > 1e-3 * scale
    np.testing.assert_allclose(out[ok], ref[ok], rtol=1e-8)


def test_fourier_K1_is_gaussian_blur():
    f = small_image()
    theta = 1.9
    g = O.spatial_taps(theta)
    w2 = np.outer(g, g)
    ref = (ndimage.correlate(f, w2, mode="constant")
           / ndimage.correlate(np.ones_like(f), w2, mode="constant"))
    np.testing.assert_allclose(O.fourier_direct(f, theta, 1, 50, [0.7]), ref,
                               rtol=1e-12)


def test_fourier_invariants():
    f = small_image()
    fitr = O.fit(255, 30.0, 5, Tmax=400)
    K, T, c = 5, fitr["T"], fitr["c"]
    out = O.fourier_direct(f, 2.0, K, T, c)
    np.testing.assert_allclose(O.fourier_direct(f.T, 2.0, K, T, c), out.T,
                               atol=1e-9)
    np.testing.assert_allclose(O.fourier_direct(f[:, ::-1], 2.0, K, T, c),
                               out[:, ::-1], atol=1e-9)
    const = np.full((12, 9), 131.0)
    np.testing.assert_allclose(O.fourier_direct(const, 2.0, K, T, c), const,
                               atol=1e-9)


def test_convergence_and_prop1_bound():
    """Error against brute force shrinks as K grows and stays inside the
    Proposition 1 bound (restated with max-norm kernel error)."""
    f = workloads.voronoi_image(96, 80, 8, False, 11)
    theta, sigma = 2.0, 30.0
    bf = O.brute_bf(f, theta, O.gaussian_range(sigma))
    Wi = O.blur_weight(*f.shape, theta)
    errs = []
    for K in (2, 3, 4, 6, 8):
        r = O.fit(255, sigma, K, Tmax=500)
        out = O.fourier_direct(f, theta, K, r["T"], r["c"])
        bound = O.prop1_bound(255, r["delta"], Wi)
        fin = np.isfinite(bound)
        assert np.all(np.abs(out - bf)[fin] <= bound[fin] + 1e-9)
        errs.append(O.psnr(bf, out))
    assert all(b > a for a, b in zip(errs, errs[1:]))
    assert errs[-1] > 90.0


def test_prop1_bound_nearly_attained():
    """The restated Proposition 1 bound is tight, not merely an upper bound:
    a pixel at 0 whose whole window sits at R meets every neighbour at the
    far end of the kernel's domain, where the fitted series' error is
    largest (|phi_hat(R) - phi(R)| = delta for these fits), and all of that
    error pulls the output one way.  The error there reaches over 3/4 of
    the bound, so a bound with a looser constant (by 4/3 or more) fails."""
    R = 255
    theta = 1.0
    rr = int(math.ceil(3 * theta))
    n = 2 * rr + 1
    f = np.full((n, n), float(R))
    f[rr, rr] = 0.0
    Wi = O.blur_weight(n, n, theta)
    for sigma, K in ((40.0, 8), (60.0, 5)):
        r = O.fit(R, sigma, K)
        t = np.arange(-R, R + 1)
        nu = 2 * np.pi / (2 * r["T"] + 1)
        phihat = sum(r["c"][k] * np.cos(nu * t * k) for k in range(K))
        err_t = np.abs(phihat - O.gaussian_range(sigma)(t))
        assert err_t[-1] == pytest.approx(r["delta"], rel=1e-9)   # worst at t = R
        bf = O.brute_bf(f, theta, O.gaussian_range(sigma))
        fo = O.fourier_direct(f, theta, K, r["T"], r["c"])
        bound = O.prop1_bound(R, r["delta"], Wi)[rr, rr]
        err = abs(fo[rr, rr] - bf[rr, rr])
        assert np.isfinite(bound) and 0.75 * bound <= err <= bound, (sigma, K, err, bound)


def test_psnr_definition():
    """Sec. III: PSNR = 10 log10(255^2 / MSE)."""
    a = np.zeros((4, 4))
    b = np.full((4, 4), 1.0)
    assert O.psnr(a, b) == pytest.approx(20 * math.log10(255.0))
    assert O.max_abs(a, b) == 1.0


def test_psnr_above_40db_at_eps_0p1():
    """Sec. III, after Table I: even at eps = 0.1 the PSNR against brute
    force stays above 40 dB (trend check on the synthetic stand-in image;
    the paper's own images are not available)."""
    f = workloads.voronoi_image(128, 128, 12, False, 12)
    theta = 3.0
    for sigma in (15.0, 30.0, 50.0):
        a = O.algorithm1(255, sigma, 0.1)
        out = O.fourier_direct(f, theta, a["K"], a["T"], a["c"])
        bf = O.brute_bf(f, theta, O.gaussian_range(sigma))
        assert O.psnr(bf, out) > 40.0


def test_row_bands_equal_the_whole_image_oracle():
    """The row-band driver (oracle/bands.py) only splits and stacks: on an
    image with ragged bands, bands thinner than the radius and an image
    shorter than the radius, its (out, N, D, W) equal the single-process
    oracle bit for bit."""
    from oracle.bands import BandPool
    rng = np.random.default_rng(3)
    cases = [(workloads.voronoi_image(150, 90, 9, True, 21), 3.0, 5, 7),
             (rng.uniform(0, 255, size=(7, 40)), 4.0, 3, 3),
             (workloads.voronoi_image(61, 33, 4, False, 22), 2.5, 13, 4)]
    with BandPool(workers=3) as pool:
        for f, theta, nbands, K in cases:
            r = O.fit(255, 30.0, K, Tmax=400)
            out, num, den = O.fourier_direct(f, theta, K, r["T"], r["c"], return_nd=True)
            b = pool.fourier_direct(f, theta, K, r["T"], r["c"], nbands=nbands)
            assert np.array_equal(b[0], out) and np.array_equal(b[1], num)
            assert np.array_equal(b[2], den)
            assert np.array_equal(b[3], O.blur_weight(*f.shape, theta))


def test_full_image_stats_on_planted_errors():
    """full_image_stats: masked count from the oracle's D/W, error maxima
    split by the mask, PSNR over all and over unmasked pixels."""
    from oracle.bands import full_image_stats
    ref = np.full((10, 10), 100.0)
    Wi = np.full((10, 10), 2.0)
    den = np.full((10, 10), 1.0)
    den[0, 0] = 0.01          # D/W = 0.005: masked
    got = ref.copy()
    got[0, 0] += 40.0         # masked pixel, large error
    got[5, 5] += 0.25
    s = full_image_stats(got, ref, den, Wi)
    assert s["masked"] == 1 and s["pixels"] == 100
    assert s["maxabs_unmasked"] == 0.25 and s["maxabs_masked"] == 40.0
    assert s["maxabs_all"] == 40.0
    assert s["psnr_unmasked_db"] == pytest.approx(10 * math.log10(255.0 ** 2 / (0.0625 / 99)))
    assert s["psnr_all_db"] == pytest.approx(10 * math.log10(255.0 ** 2 / ((1600 + 0.0625) / 100)))
