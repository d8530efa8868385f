"""fobf_filter_ws_static: the workspace form with the library's static
device scratch (for callers that cannot allocate).  Its output must equal
fobf_filter_ws's with a caller workspace bit for bit -- the same kernels
on the same inputs, only the workspace address differs -- on two calls in a
row, the second on a smaller image, and it must reject images whose
workspace exceeds the static array before any device work."""
import ctypes as C

import numpy as np
import pytest

import oracle as O
import workloads


def test_static_scratch_rejects_oversize_on_the_host():
    """An image needing more than FOBF_STATIC_SCRATCH_BYTES of workspace is
    rejected with FOBF_EINVAL from host arithmetic alone (runs without a
    GPU: no HIP call happens before the check)."""
    import paper_1811_02168_amd as F
    c = (C.c_double * 32)(0.5, 0.5)
    H, W = 4096, 8192                     # 256 MiB of N and D at theta = 10
    assert F.filter_workspace_size(H, W, 10.0, "fp32") > F.fobf.STATIC_SCRATCH_BYTES
    fake_in, fake_out = C.c_void_p(0x100000000), C.c_void_p(0x300000000)
    st = F.lib.fobf_filter_ws_static(fake_in, fake_out, H, W, W, W, 10.0, 2, 40, c,
                                     F.FP32, 0, None)
    assert st == F.fobf.EINVAL and "static scratch" in F.last_error()
    # argument errors are fobf_filter_ws's
    st = F.lib.fobf_filter_ws_static(fake_in, fake_out, 64, 64, 64, 64, 0.0, 2, 40, c,
                                     F.FP32, 0, None)
    assert st == F.fobf.EINVAL
    assert F.fobf.STATIC_SCRATCH_BYTES == 8 * 4096 * 4096


@pytest.mark.gpu
def test_static_scratch_equals_caller_workspace():
    """Two calls in a row through the C ABI: the 4096^2 benchmark image
    (theta = 10, K = 8, sigma = 50, float32: the whole 128 MiB), then a
    smaller 2600 x 2200 crop at theta = 5 in two-word fp16.  Each output
    equals fobf_filter_ws with a caller workspace bit for bit, and sampled
    pixels match the FP64 oracle (eq. (1) with the same cosine series)."""
    import torch
    import paper_1811_02168_amd as F
    base = workloads.C3.image()
    cases = [(base, 10.0, 8, 50.0, "fp32"),
             (np.ascontiguousarray(base[300:2900, 1000:3200]), 5.0, 6, 30.0, "fp16x2")]
    rng = np.random.default_rng(11)
    for f, theta, K, sigma, prec in cases:
        H, W = f.shape
        print(f"static scratch case {H}x{W} theta={theta} K={K} {prec}", flush=True)
        need = F.filter_workspace_size(H, W, theta, prec)
        assert 0 < need <= F.fobf.STATIC_SCRATCH_BYTES
        coef = F.fit(255, sigma, K, eps=1e9)
        img = torch.from_numpy(f.astype(np.float32)).cuda()
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        want = F.filter(img, theta, K, coef.T, coef.c, prec=prec, workspace=ws)
        got = torch.full_like(img, float("nan"))
        st = F.lib.fobf_filter_ws_static(C.c_void_p(img.data_ptr()), C.c_void_p(got.data_ptr()),
                                         H, W, W, W, theta, K, coef.T, F.fobf._carr(coef.c, K),
                                         F.fobf._PREC[prec], 0, F.fobf._stream_ptr(None))
        torch.cuda.synchronize()
        assert st == F.fobf.OK, F.last_error()
        assert torch.equal(got, want)
        ys, xs = rng.integers(0, H, 48), rng.integers(0, W, 48)
        ref, _, _ = O.brute_bf_points(f, theta, O.cosine_series(coef.c, coef.T), ys, xs)
        err = float(np.max(np.abs(got.cpu().numpy()[ys, xs] - ref)))
        print(f"  bit-identical to the caller-workspace call; sampled max-abs {err:.3g}")
        assert err <= 0.05
