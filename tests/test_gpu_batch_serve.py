"""GPU tests of the batched persistent launch, the autotuner table, and the
continuous-batching server.  Every result is checked against the single
image kernel and, on small cases, against the FP64 oracle."""
import threading

import numpy as np
import pytest

import oracle as O
import workloads

pytestmark = pytest.mark.gpu

TOL = 0.5


def dev_img(f):
    import torch
    return torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).cuda()


def single(F, img, theta, K, T, c, prec):
    import torch
    out = F.filter(img, theta, K, T, c, prec=prec)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def small_batch(n=18, seed=5):
    """Uneven jobs: sizes 20..300 with random aspect, theta in [0.5, 12]
    (both radius classes), K in 1..10."""
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(n):
        H = int(rng.integers(20, 300))
        W = int(rng.integers(20, 300))
        theta = float(rng.uniform(0.5, 12.0))
        sigma = float(round(rng.uniform(10, 80)))
        K = int(rng.integers(1, 11))
        f = workloads.voronoi_image(H, W, max(2, H * W // 500), True, 900 + i)
        jobs.append((f, theta, sigma, K))
    return jobs


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16", "fp16x2"])
def test_batch_matches_single(prec):
    import torch
    import paper_1811_02168_amd as F
    jobs = small_batch()
    imgs, outs, descs = [], [], []
    for f, theta, sigma, K in jobs:
        coef = F.fit(255, sigma, K, eps=1e9)
        img = dev_img(f)
        out = torch.full_like(img, -1.0)
        imgs.append(img)
        outs.append(out)
        descs.append(F.make_job(img, out, theta, K, coef.T, coef.c, prec=prec))
    F.filter_batch(descs)
    torch.cuda.synchronize()
    for (f, theta, sigma, K), img, out in zip(jobs, imgs, outs):
        coef = F.fit(255, sigma, K, eps=1e9)
        got = out.cpu().numpy().astype(np.float64)
        if prec == "fp32":
            # the batch runs the single-image kernel's tile body with the
            # job's own step count: the same sums in the same order
            ref1 = F.filter(img, theta, K, coef.T, coef.c, algo="mfma")
            torch.cuda.synchronize()
            assert np.array_equal(got, ref1.cpu().numpy().astype(np.float64)), (f.shape, theta)
            continue
        ref1 = single(F, img, theta, K, coef.T, coef.c, prec)
        d = float(np.max(np.abs(got - ref1)))
        assert d <= TOL, (f.shape, theta, K, d)
    # oracle on the first few (small enough for the FP64 oracle)
    for (f, theta, sigma, K), out in list(zip(jobs, outs))[:4]:
        coef = F.fit(255, sigma, K, eps=1e9)
        ref, num, den = O.fourier_direct(f, theta, K, coef.T, coef.c, return_nd=True)
        mask = den / O.blur_weight(*f.shape, theta) >= 0.01
        got = out.cpu().numpy().astype(np.float64)
        assert float(np.max(np.abs(got - ref)[mask])) <= (0.05 if prec == "fp32" else TOL)


def test_batch_mixed_precisions_and_edge_jobs():
    import torch
    import paper_1811_02168_amd as F
    jobs = small_batch(n=9, seed=8)
    descs, outs, refs = [], [], []     # each job keeps its tensors alive
    for i, (f, theta, sigma, K) in enumerate(jobs):
        prec = ["fp32", "fp16", "bf16", "fp16x2"][i % 4]
        coef = F.fit(255, sigma, K, eps=1e9)
        img = dev_img(f)
        out = torch.zeros_like(img)
        descs.append(F.make_job(img, out, theta, K, coef.T, coef.c, prec=prec))
        outs.append((out, prec))
        refs.append(single(F, img, theta, K, coef.T, coef.c, prec))
    # a 1x1 job and a job whose image is narrower than its radius
    tiny = dev_img(np.array([[77.0]]))
    tiny_out = torch.zeros_like(tiny)
    c1 = F.fit(255, 30.0, 4, eps=1e9)
    descs.append(F.make_job(tiny, tiny_out, 5.0, 4, c1.T, c1.c))
    F.filter_batch(descs)
    torch.cuda.synchronize()
    for (out, prec), ref in zip(outs, refs):
        d = float(np.max(np.abs(out.cpu().numpy() - ref)))
        assert d <= (1e-3 if prec == "fp32" else TOL)
    assert abs(float(tiny_out.cpu().numpy()[0, 0]) - 77.0) < 1e-3


def test_batch_random_mixed():
    """Seeded random batches (1..12 jobs, sizes up to 399^2, theta up to 16,
    K up to 16, precisions mixed within a batch, pitched buffers): every
    output against the oracle with the same (K, T, c), and nothing written
    outside the output views."""
    import torch
    import paper_1811_02168_amd as F
    precs = ["fp32", "fp16", "bf16", "fp16x2"]
    tol = {"fp32": 0.05, "fp16x2": 0.05, "fp16": TOL, "bf16": TOL}
    rng = np.random.default_rng(11)
    for b in range(16):
        n = int(rng.integers(1, 13))
        descs, keep = [], []
        for i in range(n):
            H = int(rng.integers(1, 400))
            W = int(rng.integers(1, 400))
            theta = float(rng.uniform(0.3, 16.0))
            K = int(rng.integers(1, 17))
            sigma = float(round(rng.uniform(20, 120)))
            prec = precs[int(rng.integers(0, 4))]
            pad = int(rng.integers(0, 3))
            f = workloads.voronoi_image(H, W, max(2, H * W // 300), bool(i % 2),
                                        20000 + 100 * b + i)
            fit = O.fit(255, sigma, K)
            buf = torch.zeros((H, W + pad), dtype=torch.float32, device="cuda")
            buf[:, :W] = torch.from_numpy(f.astype(np.float32))
            obuf = torch.full((H, W + pad + 2), -777.0, dtype=torch.float32, device="cuda")
            descs.append(F.make_job(buf[:, :W], obuf[:, :W], theta, K, fit["T"], fit["c"],
                                    prec=prec))
            keep.append((f, theta, K, fit["T"], fit["c"], prec, obuf, W))
        F.filter_batch(descs)
        torch.cuda.synchronize()
        for f, theta, K, T, c, prec, obuf, W in keep:
            o = obuf.cpu().numpy()
            assert np.all(o[:, W:] == -777.0), ("write outside the output view", b)
            ref, num, den = O.fourier_direct(f, theta, K, T, c, return_nd=True)
            mask = den / O.blur_weight(*f.shape, theta) >= 0.01
            err = float(np.max(np.abs(o[:, :W] - ref)[mask])) if mask.any() else 0.0
            print("random batch", b, f.shape, round(theta, 2), K, prec, err)
            assert err <= tol[prec], (b, f.shape, theta, K, prec, err)


def test_batch_c4_workload_sample():
    """A slice of the 256-image uneven workload (sizes log-uniform 64^2 ..
    2048^2): every image equals its single-image launch."""
    import torch
    import paper_1811_02168_amd as F
    js = workloads.batch_jobs(n=24)
    descs, items = [], []
    for j in js:
        f = workloads.job_image(j)
        coef = F.fit(255, j.sigma, j.K, eps=1e9)
        img = dev_img(f)
        out = torch.empty_like(img)
        descs.append(F.make_job(img, out, j.theta, j.K, coef.T, coef.c))
        items.append((img, out, j, coef))
    F.filter_batch(descs)
    torch.cuda.synchronize()
    for img, out, j, coef in items:
        ref = single(F, img, j.theta, j.K, coef.T, coef.c, "fp32")
        assert float(np.max(np.abs(out.cpu().numpy() - ref))) <= 1e-3


def test_batch_rejects_bad_calls():
    import torch
    import paper_1811_02168_amd as F
    f = dev_img(np.zeros((8, 8)))
    o = torch.empty_like(f)
    j = F.make_job(f, o, 1.0, 2, 5, [1.0, 0.0])
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(F.FobfError):
        F.filter_batch([j], workspace=small)
    bad = F.make_job(f, o, 1.0, 2, 5, [1.0, 0.0])
    bad.K = 0
    with pytest.raises(F.FobfError):
        F.filter_batch([j, bad])
    F.filter_batch([])   # no-op


def test_autotune_table_roundtrip(tmp_path):
    import paper_1811_02168_amd as F
    F.autotune("fp16", 512, 512, 6)
    a, nb = F.tune_get("fp16", 10.0)
    assert a == F.ALGO_MFMA and 1 <= nb <= 16
    p = tmp_path / "tune.txt"
    F.tune_save(p)
    F.tune_reset()
    F.tune_load(p)
    assert F.tune_get("fp16", 10.0) == (a, nb)
    # results are unchanged by the tile shape (fp32 parity still holds)
    F.autotune("fp32", 512, 512, 8)
    f = workloads.C3.image()[:300, :300]
    coef = F.fit(255, 50.0, 8, eps=1e9)
    got = single(F, dev_img(f), 10.0, 8, coef.T, coef.c, "fp32")
    ref = O.fourier_direct(f, 10.0, 8, coef.T, coef.c)
    assert float(np.max(np.abs(got - ref))) <= 0.05
    F.tune_reset()


# ------------------------------------------------------------- serving ---

def serve_requests(n=40, seed=3):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        side = int(np.exp(rng.uniform(np.log(16), np.log(400))))
        H = side
        W = int(side * rng.uniform(0.6, 1.6)) + 1
        f = workloads.voronoi_image(H, W, max(2, H * W // 600), True, 4000 + i)
        theta = float(rng.uniform(1.0, 10.0))
        sigma = float(round(rng.uniform(10, 100)))
        K = int(rng.choice([4, 6, 8]))
        prec = ["fp32", "fp16", "bf16", "fp16x2"][i % 4]
        reqs.append((f.astype(np.float32), theta, sigma, K, prec))
    return reqs


def served_coef(F, sigma, K, T):
    """The coefficients a server used for (sigma, K) given the period T it
    reports: its fit threads search the period locally (fobf_fit_warm),
    which finds the full scan's T* wherever E(K, T*) > 1e-12 and a period
    at float64's floor otherwise; the coefficients are the least-squares
    solve at that period (fobf_fit_period, the same solve)."""
    full = F.fit(255, sigma, K, eps=0.1)
    if full.E > 1e-12:
        assert T == full.T, (sigma, K, T, full.T)
    c = F.fit_period(255, sigma, K, T)
    assert c.E <= max(1e-12, full.E * (1 + 1e-9)), (sigma, K, T, c.E)
    return c


def expected(F, f, theta, sigma, K, prec, T):
    coef = served_coef(F, sigma, K, T)
    return single(F, dev_img(f), theta, K, coef.T, coef.c, prec)


def test_serve_mix_equals_alone():
    """Each result is the same whether its request ran alone or in the
    concurrent mix (two submitting threads, small budget forcing
    admission waits), within the stated tolerance."""
    import paper_1811_02168_amd as F
    reqs = serve_requests()
    budget = 6 * 400 * 700 * 8
    outs = [np.zeros_like(r[0]) for r in reqs]
    with F.Server(hbm_budget_bytes=budget, max_inflight=8, max_batch=4) as srv:
        tickets = [None] * len(reqs)

        def sub(idx):
            for i in idx:
                f, theta, sigma, K, prec = reqs[i]
                tickets[i] = srv.submit(f, outs[i], theta, sigma, K, prec=prec)

        th = [threading.Thread(target=sub, args=(range(k, len(reqs), 2),)) for k in (0, 1)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        periods = [None] * len(reqs)
        for i, t in enumerate(tickets):
            st, res = srv.poll(t, wait=True)
            periods[i] = res.T
            assert st == 0, (i, F.last_error())
            assert res.t_submit <= res.t_admit <= res.t_start <= res.t_done
            f, theta, sigma, K, prec = reqs[i]
            coef = served_coef(F, sigma, K, res.T)
            assert res.prec == F.effective_prec(prec, K, coef.T, coef.c)
        stats = srv.stats()
        assert stats["peak_bytes_inflight"] <= budget
        assert stats["peak_inflight"] <= 8
        assert stats["completed"] == len(reqs) and stats["failed"] == 0
    # alone: one request at a time through a fresh server
    with F.Server(hbm_budget_bytes=budget, max_inflight=1, max_batch=1) as srv:
        for i, (f, theta, sigma, K, prec) in enumerate(reqs):
            alone = np.zeros_like(f)
            st, _ = srv.poll(srv.submit(f, alone, theta, sigma, K, prec=prec), wait=True)
            assert st == 0
            tol = 1e-3 if prec == "fp32" else TOL
            assert float(np.max(np.abs(alone - outs[i]))) <= tol
            ref = expected(F, f, theta, sigma, K, prec, periods[i])
            assert float(np.max(np.abs(outs[i] - ref))) <= tol


def test_serve_tall_requests_run_the_workspace_form():
    """Requests tall enough for the workspace form run it (a launch of their
    own after the batch of the others): each result equals fobf_filter_ws
    on the same image with the coefficients the server used, bit for bit,
    and the small request sharing their batch equals its single launch."""
    import torch
    import paper_1811_02168_amd as F
    reqs = [(workloads.voronoi_image(2048, 2048, 200, True, 31), 5.0, 40.0, 8, "fp32"),
            (workloads.voronoi_image(2100, 2300, 200, True, 32), 8.0, 70.0, 6, "fp16x2"),
            (workloads.voronoi_image(90, 130, 20, True, 33), 4.0, 30.0, 5, "fp16")]
    outs = [np.zeros_like(r[0], dtype=np.float32) for r in reqs]
    budget = 1 << 30
    with F.Server(hbm_budget_bytes=budget, max_inflight=8, max_batch=8) as srv:
        tickets = [srv.submit(f.astype(np.float32), o, th, sg, K, prec=p)
                   for (f, th, sg, K, p), o in zip(reqs, outs)]
        res = [srv.poll(t, wait=True) for t in tickets]
        stats = srv.stats()
    assert stats["peak_bytes_inflight"] <= budget and stats["failed"] == 0
    for (f, theta, sigma, K, prec), o, (st, r) in zip(reqs, outs, res):
        assert st == 0, F.last_error()
        coef = served_coef(F, sigma, K, r.T)
        H, W = f.shape
        n = F.filter_workspace_size(H, W, theta, prec)
        img = dev_img(f)
        if H >= 2048:
            assert n > 0
            ws = torch.empty(n, dtype=torch.uint8, device="cuda")
            want = F.filter(img, theta, K, coef.T, coef.c, prec=prec, workspace=ws)
            torch.cuda.synchronize()
            assert np.array_equal(o, want.cpu().numpy()), (H, W, prec)
        else:
            assert n == 0
            ref = single(F, img, theta, K, coef.T, coef.c, prec)
            assert float(np.max(np.abs(o - ref))) <= TOL


def test_serve_against_oracle_small():
    import paper_1811_02168_amd as F
    f = workloads.C1.image()[:120, :150].astype(np.float32)
    out = np.zeros_like(f)
    with F.Server(hbm_budget_bytes=1 << 26) as srv:
        st, res = srv.poll(srv.submit(f, out, 3.0, 30.0, 4), wait=True)
    assert st == 0
    coef = served_coef(F, 30.0, 4, res.T)
    ref = O.fourier_direct(f.astype(np.float64), 3.0, 4, coef.T, coef.c)
    assert float(np.max(np.abs(out - ref))) <= 0.05


def test_serve_faults_and_errors():
    import paper_1811_02168_amd as F
    f = workloads.C1.image()[:64, :64].astype(np.float32)
    with F.Server(hbm_budget_bytes=1 << 24, max_inflight=1, max_batch=1) as srv:
        srv.inject_fault(1)
        o1, o2 = np.zeros_like(f), np.zeros_like(f)
        t1 = srv.submit(f, o1, 2.0, 30.0, 4)
        st1, _ = srv.poll(t1, wait=True)
        assert st1 == F.fobf.EHIP            # injected failure reported
        t2 = srv.submit(f, o2, 2.0, 30.0, 4)
        st2, _ = srv.poll(t2, wait=True)
        assert st2 == 0                      # and the server keeps serving
        with pytest.raises(F.FobfError) as e:
            srv.submit(f, o2, -1.0, 30.0, 4)
        assert e.value.status == F.fobf.EINVAL
        big = np.zeros((2048, 2048), dtype=np.float32)
        with pytest.raises(F.FobfError) as e:
            srv.submit(big, big.copy(), 2.0, 30.0, 4)
        assert e.value.status == F.fobf.ENOMEM
        with pytest.raises(F.FobfError):
            srv.poll(987654321)
        assert srv.stats()["failed"] == 1


def test_serve_destroy_with_pending():
    import paper_1811_02168_amd as F
    f = workloads.C2.image()[:256, :256].astype(np.float32)
    outs = [np.zeros_like(f) for _ in range(12)]
    srv = F.Server(hbm_budget_bytes=1 << 22, max_inflight=1, max_batch=1)
    for o in outs:
        srv.submit(f, o, 5.0, 30.0, 6)
    srv.close()                              # must not hang or fault


def test_serve_cold_fits_do_not_block_ready_requests():
    """With an empty fit cache, a request whose (sigma, K) must first be
    fitted on the host does not hold up a later request whose coefficients
    are ready; every result still equals its single-image launch."""
    import paper_1811_02168_amd as F
    f = workloads.C1.image()[:96, :112].astype(np.float32)
    F.fit_cache_clear()
    F.fit(255, 40.0, 4, eps=0.1)                     # ready key
    slow = (255, 47.0, 32)                           # K = 32: the slowest fit
    o_slow, o_fast = np.zeros_like(f), np.zeros_like(f)
    with F.Server(hbm_budget_bytes=1 << 26, max_inflight=4, max_batch=4) as srv:
        # warm the server's own table with the ready key
        st, _ = srv.poll(srv.submit(f, np.zeros_like(f), 2.0, 40.0, 4), wait=True)
        assert st == 0
        t1 = srv.submit(f, o_slow, 2.0, slow[1], slow[2])
        t2 = srv.submit(f, o_fast, 2.0, 40.0, 4)
        st2, r2 = srv.poll(t2, wait=True)
        st1, r1 = srv.poll(t1, wait=True)
    assert st1 == 0 and st2 == 0
    assert r2.t_admit <= r1.t_admit          # passed over while fitting
    c_slow = served_coef(F, slow[1], slow[2], r1.T)
    ref = single(F, dev_img(f), 2.0, slow[2], c_slow.T, c_slow.c, "fp32")
    assert float(np.max(np.abs(o_slow - ref))) <= 1e-3
    c4 = F.fit(255, 40.0, 4, eps=0.1)
    ref = single(F, dev_img(f), 2.0, 4, c4.T, c4.c, "fp32")
    assert float(np.max(np.abs(o_fast - ref))) <= 1e-3


def test_serve_many_cold_keys():
    """Twenty distinct (sigma, K) keys, none cached: all complete, each with
    the period the host fit chooses, and equal to the single-image launch."""
    import paper_1811_02168_amd as F
    F.fit_cache_clear()
    f = workloads.C1.image()[:80, :72].astype(np.float32)
    keys = [(float(s), K) for s in (12, 23, 35, 61, 88) for K in (3, 5, 7, 9)]
    outs = [np.zeros_like(f) for _ in keys]
    with F.Server(hbm_budget_bytes=1 << 26, max_inflight=6, max_batch=3) as srv:
        ts = [srv.submit(f, o, 3.0, s, K) for o, (s, K) in zip(outs, keys)]
        res = [srv.poll(t, wait=True) for t in ts]
    img = dev_img(f)
    for (st, r), o, (s, K) in zip(res, outs, keys):
        assert st == 0
        c = served_coef(F, s, K, r.T)
        ref = single(F, img, 3.0, K, c.T, c.c, "fp32")
        assert float(np.max(np.abs(o - ref))) <= 1e-3


def test_serve_coefficient_row_ordering_across_lanes():
    """Regression test of the coefficient-row ordering rule: a key's device
    row is uploaded on the lane of its first batch, queued behind that
    lane's earlier work (two 4096^2 requests keep two lanes busy), while
    later batches with the same new key run on an idle lane.  Each of those
    must wait for the upload: every output equals, bit for bit, the launch
    the server runs for its request -- the workspace form where it is used,
    else the single-image batch launch (a read of the row before it lands
    gives garbage or NaN)."""
    import torch
    import paper_1811_02168_amd as F
    def pinned(a):
        # pinned host buffers: the copies stay asynchronous, so the
        # scheduler never waits for a busy lane before issuing the next batch
        t = torch.empty(a.shape, dtype=torch.float32, pin_memory=True).numpy()
        t[:] = a
        return t

    big = pinned(workloads.C3.image())
    small = [pinned(workloads.C2.image()[64 * i:64 * i + 200, 32 * i:32 * i + 230])
             for i in range(8)]
    key_a, key_b = (43.0, 5), (57.0, 7)          # keys no other test uses
    F.fit_cache_clear()
    reqs = [(big, 4.0, key_a), (big, 4.0, key_a), (small[0], 3.0, key_a)]
    reqs += [(small[i], 2.5 + 0.25 * i, key_b) for i in range(1, 8)]
    outs = [pinned(np.full(f.shape, np.nan)) for f, _, _ in reqs]
    with F.Server(hbm_budget_bytes=8 << 30, max_inflight=16, max_batch=1) as srv:
        ts = [srv.submit(f, o, theta, s, K) for (f, theta, (s, K)), o in zip(reqs, outs)]
        res = [srv.poll(t, wait=True) for t in ts]
    for i, ((f, theta, (s, K)), o, (st, r)) in enumerate(zip(reqs, outs, res)):
        assert st == 0, (i, F.last_error())
        coef = served_coef(F, s, K, r.T)
        img = dev_img(f)
        n = F.filter_workspace_size(f.shape[0], f.shape[1], theta, "fp32")
        if n > 0:
            ws = torch.empty(n, dtype=torch.uint8, device="cuda")
            ref = F.filter(img, theta, K, coef.T, coef.c, workspace=ws)
        else:
            ref = torch.full_like(img, -1.0)
            F.filter_batch([F.make_job(img, ref, theta, K, coef.T, coef.c)])
        torch.cuda.synchronize()
        ref = ref.cpu().numpy()
        assert np.all(np.isfinite(o)), i
        assert np.array_equal(o, ref), (i, float(np.nanmax(np.abs(o - ref))))


def test_instruction_rate_probes_are_plausible():
    """fobf_peak: every measured rate is positive and within 10% above the
    published MI355X figure for its class (the matrix peaks are dense)."""
    import paper_1811_02168_amd as F
    published = {"valu_fma_f32": 157.3, "valu_sin_f32": 157.3 / 2, "mfma_f32": 157.3,
                 "mfma_f16": 2500.0, "mfma_bf16": 2500.0}
    for kind, peak in published.items():
        rate = F.peak(kind)
        print("peak", kind, rate)
        assert 0.0 < rate <= 1.1 * peak, (kind, rate)
    assert F.peak("mfma_f32") > 0.5 * 157.3


def test_batch_and_serve_run_crude_fp16_series_as_two_word():
    """fp16 staging of a series with negative lobes (K = 2, sigma = 34)
    runs as two-word fp16 in the batch launch and in the server too
    (fobf_effective_prec): the fp16 job equals the same job asked for in
    two-word fp16 bit for bit, a well-fitted fp16 job in the same batch
    keeps single-word staging, and the server reports the precision each
    request ran in."""
    import torch
    import paper_1811_02168_amd as F
    f = workloads.voronoi_image(300, 280, 280, True, 9083).astype(np.float32)
    crude = F.fit(255, 34.0, 2, eps=1e9)
    good = F.fit(255, 50.0, 8, eps=1e9)
    assert F.effective_prec("fp16", 2, crude.T, crude.c) == F.FP16X2_STAGE
    assert F.effective_prec("fp16", 8, good.T, good.c) == F.FP16_STAGE
    img = dev_img(f)
    specs = [(crude, 2, "fp16"), (crude, 2, "fp16x2"), (good, 8, "fp16"), (good, 8, "fp16x2")]
    outs = [torch.full_like(img, -1.0) for _ in specs]
    descs = [F.make_job(img, o, 3.0, K, cf.T, cf.c, prec=p) for (cf, K, p), o in zip(specs, outs)]
    F.filter_batch(descs)
    torch.cuda.synchronize()
    o = [x.cpu().numpy() for x in outs]
    assert np.array_equal(o[0], o[1])
    assert not np.array_equal(o[2], o[3])          # single-word staging kept
    ref, num, den = O.fourier_direct(f.astype(np.float64), 3.0, 2, crude.T, crude.c,
                                     return_nd=True)
    keep = den / O.blur_weight(*f.shape, 3.0) >= 0.01
    assert float(np.max(np.abs(o[0] - ref)[keep])) <= 0.05
    with F.Server(hbm_budget_bytes=1 << 28, max_inflight=4, max_batch=1) as srv:
        res = []
        for K, sigma, p in ((2, 34.0, "fp16"), (8, 50.0, "fp16"), (2, 34.0, "fp32")):
            got = np.full_like(f, np.nan)
            st, r = srv.poll(srv.submit(f, got, 3.0, sigma, K, prec=p), wait=True)
            assert st == 0, F.last_error()
            res.append((r.prec, got))
    assert [p for p, _ in res] == [F.FP16X2_STAGE, F.FP16_STAGE, F.FP32]
    assert np.array_equal(res[0][1], o[0])


def test_serve_cancel_and_deadline():
    """fobf_serve_cancel and the per-request admission deadline: with one
    request in flight at a time, a request queued behind a 4096^2 one can be
    cancelled (ECANCELED, never runs), a request whose deadline passes
    before it is admitted completes with ETIMEDOUT, one with a generous
    deadline completes normally, and a request already on the device cannot
    be cancelled (EBUSY, or EINVAL once it has completed)."""
    import paper_1811_02168_amd as F

    def pinned(a):
        import torch
        t = torch.empty(a.shape, dtype=torch.float32, pin_memory=True).numpy()
        t[:] = a
        return t

    big = pinned(workloads.C3.image())
    big_out = pinned(np.zeros(big.shape))
    small = workloads.C1.image()[:64, :80].astype(np.float32)
    outs = [np.full(small.shape, -1.0, dtype=np.float32) for _ in range(3)]
    with F.Server(hbm_budget_bytes=4 << 30, max_inflight=1, max_batch=1) as srv:
        srv.poll(srv.submit(small, outs[2], 3.0, 40.0, 4), wait=True)   # fit the key
        t_big = srv.submit(big, big_out, 10.0, 40.0, 4)
        t_c = srv.submit(small, outs[0], 3.0, 40.0, 4)
        t_late = srv.submit(small, outs[1], 3.0, 40.0, 4, deadline_s=1e-4)
        t_ok = srv.submit(small, outs[2], 3.0, 40.0, 4, deadline_s=30.0)
        assert srv.cancel(t_c) == F.fobf.OK
        st_c, r_c = srv.poll(t_c, wait=True)
        st_late, _ = srv.poll(t_late, wait=True)
        st_ok, _ = srv.poll(t_ok, wait=True)
        try:
            busy = srv.cancel(t_big)
        except F.FobfError as e:
            busy = e.status
        st_big, _ = srv.poll(t_big, wait=True)
        stats = srv.stats()
    assert st_c == F.fobf.ECANCELED and r_c.t_done >= r_c.t_submit
    assert np.all(outs[0] == -1.0)                   # never ran
    assert st_late == F.fobf.ETIMEDOUT and np.all(outs[1] == -1.0)
    assert st_ok == 0 and st_big == 0
    assert busy in (F.fobf.EBUSY, F.fobf.EINVAL)
    assert stats["failed"] == 2 and stats["completed"] == stats["submitted"] == 5
    coef = F.fit(255, 40.0, 4, eps=0.1)
    ref = O.fourier_direct(small.astype(np.float64), 3.0, 4, coef.T, coef.c)
    assert float(np.max(np.abs(outs[2] - ref))) <= 0.05
