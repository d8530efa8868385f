"""GPU runs of the debug-check build (libfobf_check.so, compiled with
FOBF_CHECKS=1).  Its kernels fill their LDS with NaN words before use, so a
read of LDS they never wrote would reach the output, and check their
indices as they run: LDS, image, workspace and output accesses inside their
extents, every non-zero tap met inside its output's window, every vertical
ring slot holding the block its taps are for, every batch tile inside its
job.  Each case runs every entry point of the filter (LDS form in all four
precisions and the vector path, workspace form in all four, the
static-scratch entry, a mixed batch) through the check build: no violation
may be recorded, and the output must equal the release build's: bit for bit
in float32 and single-word fp16 (the checks only read, so the arithmetic is
the same); in the two-word modes within a fifth of their parity bound,
since the compiler may turn a split's subtract-and-round into one
mixed-precision instruction in one build and not the other (measured up to
3e-3 levels, at a crude K = 2 series whose small D/W magnifies it)."""
import os
import tempfile

import numpy as np
import pytest

import oracle as O
import workloads

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "fp16", "bf16", "fp16x2"]
# largest |check build - release build| allowed per precision
SAME = {"fp32": 0.0, "fp16": 0.0, "bf16": 0.1, "fp16x2": 0.01}


@pytest.fixture(scope="module")
def libs():
    import paper_1811_02168_amd as F
    from paper_1811_02168_amd import fobf as M
    rel = M.lib
    chk = F.load_check_library()
    # both builds pick their tile heights from their own tuning tables:
    # start both from the built-in defaults, and give the release build its
    # table back afterwards
    path = os.path.join(tempfile.mkdtemp(), "tune.txt")
    assert rel.fobf_tune_save(path.encode()) == 0
    assert rel.fobf_tune_reset() == 0 and chk.fobf_tune_reset() == 0
    assert F.check_take(chk) == 0
    yield M, rel, chk
    M.lib = rel
    with open(path) as fh:
        rows = [ln for ln in fh if ln.strip() and not ln.startswith("#")]
    assert (rel.fobf_tune_load(path.encode()) if rows else rel.fobf_tune_reset()) == 0


def through(M, lib, fn):
    """Runs fn() with the binding's calls going to `lib`."""
    import torch
    saved = M.lib
    M.lib = lib
    try:
        out = fn()
        torch.cuda.synchronize()
        return out
    finally:
        M.lib = saved


def bits_equal(a, b):
    import torch
    return torch.equal(a.contiguous().view(torch.int32), b.contiguous().view(torch.int32))


def names(bits):
    import paper_1811_02168_amd as F
    return [k for k, v in F.CHECK_BITS.items() if bits & v]


def image(H, W, seed, pad=0):
    import torch
    f = workloads.voronoi_image(H, W, max(4, int(np.sqrt(H * W) / 16)), True, seed)
    buf = torch.zeros((H, W + pad), dtype=torch.float32, device="cuda")
    buf[:, :W] = torch.from_numpy(f.astype(np.float32))
    return buf[:, :W]


def fitted(sigma, K):
    r = O.fit(255, sigma, K)
    return r["T"], r["c"]


def used(prec, K, T, c):
    """The precision the call runs in (fp16 staging of a crude series runs
    as two-word fp16)."""
    import paper_1811_02168_amd as F
    return PRECS[F.effective_prec(prec, K, T, c)]


def agree(got, want, prec, case):
    import torch
    if SAME[prec] == 0.0:
        assert bits_equal(got, want), (case, float((got - want).abs().nan_to_num(1e30).max()))
    else:
        assert torch.equal(torch.isfinite(got), torch.isfinite(want)), case
        fin = torch.isfinite(want)
        d = float((got[fin] - want[fin]).abs().max()) if bool(fin.any()) else 0.0
        assert d <= SAME[prec], (case, d)


def compare(libs, case, call, prec=None, parts=None):
    """call() -> output tensor; run it through both builds, check that the
    check build recorded nothing and that the outputs agree (per part:
    [(numel, prec)] for a concatenation of several outputs)."""
    import paper_1811_02168_amd as F
    M, rel, chk = libs
    want = through(M, rel, call)
    got = through(M, chk, call)
    bits = F.check_take(chk)
    print(case, "violations:", names(bits), flush=True)
    assert bits == 0, (case, names(bits))
    if parts is None:
        parts = [(want.numel(), prec)]
    got, want = got.reshape(-1), want.reshape(-1)
    o = 0
    for n, p in parts:
        agree(got[o:o + n], want[o:o + n], p, case)
        o += n


# (H, W, theta, K, sigma, pitch pad): single pixels, ragged edges, every
# radius class of the LDS form up to r = 48, pitched rows
LDS_CASES = [
    (1, 1, 1.0, 3, 30.0, 0),
    (7, 5, 2.0, 1, 20.0, 0),
    (300, 517, 5.0, 8, 40.0, 0),
    (129, 1000, 10.0, 3, 60.0, 0),
    (333, 200, 16.0, 8, 50.0, 0),
    (200, 301, 3.0, 4, 25.0, 37),
    (97, 161, 13.0, 7, 80.0, 5),
]


@pytest.mark.parametrize("case", LDS_CASES, ids=lambda c: "x".join(map(str, c[:3])))
def test_checked_lds_form(libs, case):
    import paper_1811_02168_amd as F
    H, W, theta, K, sigma, pad = case
    T, c = fitted(sigma, K)
    img = image(H, W, 11 + H, pad)
    for prec in PRECS:
        compare(libs, ("filter", case, prec),
                lambda: F.filter(img, theta, K, T, c, prec=prec, algo="mfma"),
                used(prec, K, T, c))
    compare(libs, ("filter valu", case),
            lambda: F.filter(img, theta, K, T, c, prec="fp32", algo="valu"), "fp32")


# tall enough for the workspace form (tiles of at least 8 blocks); radius
# classes DV = 2 .. 6 and the fp16 two-frequency groups at K = 1, 2, 7
WS_CASES = [
    (2600, 3000, 7.0, 8, 25.0),
    (4100, 2049, 10.0, 7, 50.0),
    (3001, 1500, 2.5, 2, 60.0),
    (2048, 4096, 13.0, 1, 40.0),
]


@pytest.mark.parametrize("case", WS_CASES, ids=lambda c: "x".join(map(str, c[:3])))
def test_checked_workspace_form(libs, case):
    import torch
    import paper_1811_02168_amd as F
    H, W, theta, K, sigma = case
    T, c = fitted(sigma, K)
    img = image(H, W, 5 + W)
    for prec in PRECS:
        n = F.filter_workspace_size(H, W, theta, prec)
        # (float32 below r = 14 runs the LDS form: no workspace used)
        assert n > 0 or (prec == "fp32" and np.ceil(3 * theta) < 14), (case, prec)
        ws = torch.full((max(n, 16) // 4,), float("nan"), dtype=torch.float32, device="cuda")
        compare(libs, ("filter_ws", case, prec),
                lambda: F.filter(img, theta, K, T, c, prec=prec, workspace=ws),
                used(prec, K, T, c))
    out = torch.empty_like(img)
    compare(libs, ("filter_ws_static", case),
            lambda: F.filter_ws_static(img, theta, K, T, c, prec="fp32", out=out).clone(),
            "fp32")


def test_checked_batch(libs):
    import torch
    import paper_1811_02168_amd as F
    rng = np.random.default_rng(77)
    jobs_spec = []
    # every precision in every radius class (r <= 24, r <= 32, r <= 48)
    for i, theta in enumerate([1.5, 4.0, 8.0, 10.0, 15.0, 2.5, 6.0, 12.0]):
        for prec in PRECS:
            H = int(rng.integers(1, 700))
            W = int(rng.integers(1, 700))
            K = int(rng.integers(1, 10))
            sigma = float(rng.integers(15, 90))
            jobs_spec.append((H, W, theta, K, sigma, prec, 100 * i + len(jobs_spec)))
    imgs = [image(H, W, seed) for (H, W, _, _, _, _, seed) in jobs_spec]
    coefs = [fitted(s, K) for (_, _, _, K, s, _, _) in jobs_spec]

    def call():
        outs = [torch.full_like(im, -1.0) for im in imgs]
        jobs = [F.make_job(im, o, spec[2], spec[3], T, c, prec=spec[5])
                for im, o, spec, (T, c) in zip(imgs, outs, jobs_spec, coefs)]
        F.filter_batch(jobs)
        torch.cuda.synchronize()
        return torch.cat([o.reshape(-1) for o in outs])

    compare(libs, ("batch", len(jobs_spec)), call,
            parts=[(im.numel(), used(spec[5], spec[3], T, c))
                   for im, spec, (T, c) in zip(imgs, jobs_spec, coefs)])
