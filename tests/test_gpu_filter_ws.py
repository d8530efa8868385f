"""GPU parity of fobf_filter_ws, the workspace form of the filter (each
tile's N and D in a caller-provided device workspace, tiles up to 512 rows
tall; float32 also stages its channels per workgroup): float32 and the
two-word modes against the FP64 oracle with the same (K, T, c), against the
LDS form (bit for bit in float32: the same sums in the same order), at
ragged and pitched sizes of every radius class it covers, in a captured
graph, and with a reused workspace."""
import numpy as np
import pytest

import oracle as O
import workloads

pytestmark = pytest.mark.gpu

TOL = {"fp32": 0.05, "fp16x2": 0.05, "bf16": 0.5, "fp16": 0.5}
WS_PRECS = ["fp32", "fp16", "bf16", "fp16x2"]


def dv_of(theta):
    r = int(np.ceil(3 * theta))
    return (16 + 2 * r + 15) // 16


def fitted(sigma, K):
    r = O.fit(255, sigma, K)
    return r["T"], r["c"]


def points(H, W, n, seed):
    rng = np.random.default_rng(seed)
    ys = list(rng.integers(0, H, n))
    xs = list(rng.integers(0, W, n))
    for y in (0, 1, 30, 255, 256, 511, 512, H // 2, H - 31, H - 1):
        for x in (0, 1, 127, 128, W // 2, W - 1):
            ys.append(min(y, H - 1))
            xs.append(min(x, W - 1))
    return np.array(ys), np.array(xs)


def run_ws(f, theta, K, T, c, prec, pad=0):
    """fobf_filter_ws on f (pitched by pad columns); returns the output and
    whether the workspace form was used."""
    import torch
    import paper_1811_02168_amd as F
    H, W = f.shape
    buf = torch.zeros((H, W + pad), dtype=torch.float32, device="cuda")
    buf[:, :W] = torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32))
    obuf = torch.full((H, W + pad + 3), -777.0, dtype=torch.float32, device="cuda")
    n = F.filter_workspace_size(H, W, theta, prec)
    ws = torch.empty(max(n, 1), dtype=torch.uint8, device="cuda")
    F.filter(buf[:, :W], theta, K, T, c, prec=prec, out=obuf[:, :W], workspace=ws)
    torch.cuda.synchronize()
    o = obuf.cpu().numpy()
    assert np.all(o[:, W:] == -777.0), "write outside the output view"
    return o[:, :W].astype(np.float64), n > 0


@pytest.mark.parametrize("prec", WS_PRECS)
def test_ws_c3_full_size_sampled(prec):
    """4096^2, theta = 10, K = 8 (the benchmark image): sampled outputs of
    the workspace form against eq. (1) with the fitted cosine series."""
    cfg = workloads.C3
    f = cfg.image()
    for sigma in cfg.sigmas:
        T, c = fitted(sigma, cfg.K)
        got, used = run_ws(f, cfg.theta, cfg.K, T, c, prec)
        assert used
        ys, xs = points(*f.shape, 500, int(sigma) + 3)
        ref, num, den = O.brute_bf_points(f, cfg.theta, O.cosine_series(c, T), ys, xs)
        err = np.abs(got[ys, xs] - ref)
        print("ws C3", prec, sigma, float(err.max()))
        assert float(err.max()) <= TOL[prec]


# (H, W, theta, K, sigma, pad): every radius class of the workspace form
# (DV = 2 .. 6), ragged tile edges, pitched buffers
SHAPES = [
    (2048, 2048, 1.5, 6, 30.0, 0),     # r = 5, DV = 2
    (2500, 2100, 5.0, 6, 40.0, 3),     # r = 15, DV = 3
    (2600, 3000, 7.0, 8, 25.0, 1),     # r = 21, DV = 4
    (4100, 2049, 10.0, 8, 50.0, 2),    # r = 30, DV = 5
    (3001, 1500, 12.0, 5, 60.0, 0),    # r = 36, DV = 6
    (2048, 2300, 4.0, 32, 12.0, 1),    # r = 12, DV = 3, the largest order
]


@pytest.mark.parametrize("prec", WS_PRECS)
@pytest.mark.parametrize("H,W,theta,K,sigma,pad", SHAPES)
def test_ws_shapes_against_oracle_and_lds_form(prec, H, W, theta, K, sigma, pad):
    import torch
    import paper_1811_02168_amd as F
    f = workloads.voronoi_image(H, W, max(4, H * W // 65536), True, H + 7 * W)
    T, c = fitted(sigma, K)
    got, used = run_ws(f, theta, K, T, c, prec, pad=pad)
    # float32 takes the workspace form from r = 14 on (below, the call is
    # the LDS form)
    assert used == (prec != "fp32" or int(np.ceil(3 * theta)) >= 14)
    ys, xs = points(H, W, 300, H * 3 + W)
    ref, num, den = O.brute_bf_points(f, theta, O.cosine_series(c, T), ys, xs)
    mask = den / O.blur_weight(H, W, theta)[ys, xs] >= 0.01
    err = np.abs(got[ys, xs] - ref)[mask]
    # the LDS form on the same image: both within the bound of the exact
    # result, hence within twice it of each other
    lds = F.filter(torch.from_numpy(f.astype(np.float32)).cuda(), theta, K, T, c, prec=prec)
    d = float(np.max(np.abs(lds.cpu().numpy() - got)))
    print("ws shape", prec, H, W, theta, K, float(err.max()), "vs lds", d)
    assert float(err.max()) <= TOL[prec]
    assert d <= 2 * TOL[prec]
    if prec == "fp32":
        assert d == 0.0


def test_ws_falls_back_where_not_used():
    """Short or narrow images and the largest radius class need no
    workspace: fobf_filter_ws then equals fobf_filter bit for bit."""
    import torch
    import paper_1811_02168_amd as F
    cases = [(4096, 512, 10.0, "fp32"), (1024, 2048, 5.0, "fp16"),
             (600, 700, 5.0, "fp16x2"), (2048, 2048, 15.0, "bf16"),
             (2048, 2048, 3.0, "fp32")]
    for H, W, theta, prec in cases:
        assert F.filter_workspace_size(H, W, theta, prec) == 0
        f = workloads.voronoi_image(H, W, 64, True, 31 + H)
        T, c = fitted(40.0, 6)
        img = torch.from_numpy(f.astype(np.float32)).cuda()
        a = F.filter(img, theta, 6, T, c, prec=prec)
        b = F.filter(img, theta, 6, T, c, prec=prec,
                     workspace=torch.empty(16, dtype=torch.uint8, device="cuda"))
        torch.cuda.synchronize()
        assert torch.equal(a, b), (H, W, theta, prec)


def test_ws_reused_workspace_and_errors():
    """One workspace serves a large call, then a smaller one (no clearing
    needed: every tile writes its N and D before reading them); a short
    workspace is rejected before any launch."""
    import torch
    import paper_1811_02168_amd as F
    cfg = workloads.C3
    f = cfg.image()
    T, c = fitted(50.0, cfg.K)
    img = torch.from_numpy(f.astype(np.float32)).cuda()
    n = F.filter_workspace_size(4096, 4096, cfg.theta, "fp16x2")
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    ws.fill_(0xFF)                        # NaN patterns: must never be read
    big = F.filter(img, cfg.theta, cfg.K, T, c, prec="fp16x2", workspace=ws)
    sub = img[:2048, 1000:3048]
    small = F.filter(sub, cfg.theta, cfg.K, T, c, prec="fp16x2", workspace=ws)
    ref_big = F.filter(img, cfg.theta, cfg.K, T, c, prec="fp16x2")
    ref_small = F.filter(sub, cfg.theta, cfg.K, T, c, prec="fp16x2")
    torch.cuda.synchronize()
    assert torch.isfinite(big).all() and torch.isfinite(small).all()
    assert float((big - ref_big).abs().max()) <= 2 * TOL["fp16x2"]
    assert float((small - ref_small).abs().max()) <= 2 * TOL["fp16x2"]
    with pytest.raises(F.FobfError):
        F.filter(img, cfg.theta, cfg.K, T, c, prec="fp16x2", workspace=ws[: n - 256])
    with pytest.raises(ValueError):
        F.filter(img, cfg.theta, cfg.K, T, c, prec="fp16x2",
                 workspace=torch.empty(n, dtype=torch.uint8))


def test_ws_in_a_captured_graph():
    """fobf_filter_ws enqueues kernels only: captured once, replayed three
    times with new input written eagerly between replays, every replay
    equals the eager call bit for bit."""
    import torch
    import paper_1811_02168_amd as F
    f = workloads.voronoi_image(2048, 2048, 64, True, 77).astype(np.float32)
    T, c = fitted(30.0, 6)
    theta = 5.0
    img = torch.from_numpy(f).cuda()
    outs, wss = {}, {}
    for p in WS_PRECS:
        outs[p] = torch.empty_like(img)
        wss[p] = torch.empty(F.filter_workspace_size(2048, 2048, theta, p),
                             dtype=torch.uint8, device="cuda")
        F.filter(img, theta, 6, T, c, prec=p, out=outs[p], workspace=wss[p])
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for p in WS_PRECS:
            F.filter(img, theta, 6, T, c, prec=p, out=outs[p], workspace=wss[p])
    for rep in range(3):
        img.copy_(torch.from_numpy(np.roll(f, 29 * rep, axis=0)).cuda())
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for p in WS_PRECS:
            ref = F.filter(img, theta, 6, T, c, prec=p,
                           workspace=torch.empty_like(wss[p]))
            torch.cuda.synchronize()
            assert torch.equal(outs[p], ref), (rep, p)


def test_ws_fp32_bitwise_random():
    """float32 through fobf_filter_ws computes the same sums in the same
    order as fobf_filter: seeded random large images (sizes, radius classes
    DV = 2..6, orders, pitched buffers) give bit-identical outputs."""
    import torch
    import paper_1811_02168_amd as F
    rng = np.random.default_rng(515)
    used = 0
    for case in range(16):
        H = int(rng.integers(1900, 4400))
        W = int(rng.integers(1000, 4400))
        theta = float(rng.uniform(4.4, 13.3))    # float32 takes the form from r = 14
        K = int(rng.integers(1, 17))
        sigma = float(round(rng.uniform(15, 120)))
        pad = int(rng.integers(0, 5))
        f = workloads.voronoi_image(H, W, max(4, H * W // 60000), bool(case % 2), 40000 + case)
        T, c = fitted(sigma, K)
        got, ws_used = run_ws(f, theta, K, T, c, "fp32", pad=pad)
        used += ws_used
        ref = F.filter(torch.from_numpy(f.astype(np.float32)).cuda(), theta, K, T, c,
                       prec="fp32")
        torch.cuda.synchronize()
        print("fp32 ws bitwise", case, H, W, round(theta, 2), K, ws_used)
        assert np.array_equal(got, ref.cpu().numpy().astype(np.float64)), (case, H, W, theta)
    assert used >= 10


@pytest.mark.parametrize("K", [1, 2, 3, 4, 7, 16, 32])
def test_ws_fp16_every_group_shape(K):
    """The fp16 workspace form folds channel groups two frequencies at a
    time ({f, 1}, {2, 3}, .., a last single frequency when K is even, {f}
    alone when K = 1).  Every one of those shapes on a 2048^2 image at
    theta = 10 against eq. (1) with the same cosine series at sampled
    pixels.  The series is the normalised Fejer kernel (non-negative, so
    single-word fp16 staging is kept: fobf_effective_prec)."""
    import paper_1811_02168_amd as F
    H = W = 2048
    theta, T = 10.0, 200
    c = np.array([1.0 / K] + [2.0 * (1.0 - k / K) / K for k in range(1, K)])
    assert F.effective_prec("fp16", K, T, c) == F.FP16_STAGE
    f = workloads.voronoi_image(H, W, 64, True, 77 + K)
    got, used = run_ws(f, theta, K, T, c, "fp16")
    assert used
    ys, xs = points(H, W, 300, 5 + K)
    ref, num, den = O.brute_bf_points(f, theta, O.cosine_series(c, T), ys, xs)
    mask = den / O.blur_weight(H, W, theta)[ys, xs] >= 0.01
    err = float(np.max(np.abs(got[ys, xs] - ref)[mask]))
    print("ws fp16 groups K", K, err)
    assert err <= TOL["fp16"]
