#!/usr/bin/env python3
"""Benchmark of the Fourier bilateral filter on one MI355X.

Workload (the configuration the headline metric is quoted on): one
4096x4096 synthetic 8-bit-like image (Voronoi + ramp + noise, 256 cells,
seed 1003), theta = 10 (61-tap truncated Gaussian), K = 8, R = 255, and the
three range widths sigma = 20, 50, 100.  One step is the whole hot path for
all three sigmas: host fit lookup (float64, cached), coefficient upload in
the kernel arguments, and the fused filter kernel.  Inputs are resident in
HBM before timing starts.

`value` is the float32 ("plain") throughput; the staged ("mixed") forms --
fp16, two-word bf16 and two-word fp16 -- are timed the same way and
reported under "mixed", each with its max-abs and PSNR against the FP64
oracle on sampled pixels.

Prints ONE JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X dense fp32 (vector and matrix)
PEAK_HBM_GBS = 8000.0
FLOP_PER_PX = None            # set from theta, K: 4 (2r+1)(4K-3)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-images", type=int, default=256)
    ap.add_argument("--serve-requests", type=int, default=4000,
                    help="timed requests of the warm-cache serving leg (after "
                    "a tenth as many warm-up requests); the cold-cache leg "
                    "times a quarter as many")
    ap.add_argument("--modes",
                    default="fp32,fp32_ws,fp32_valu,fp16,fp16_ws,bf16,fp16x2,bf16_ws,fp16x2_ws",
                    help="precisions; a _ws suffix calls fobf_filter_ws with a workspace, "
                    "fp32_valu the vector-ALU kernel")
    ap.add_argument("--profile-run", action="store_true",
                    help="for rocprofv3 counter passes: one 256 MiB device "
                    "copy (calibrates FETCH_SIZE/WRITE_SIZE), then one launch "
                    "per precision of the C3 filter at sigma=50, then exit")
    ap.add_argument("--write-traffic", metavar="DIR",
                    help="turn the FETCH_SIZE / WRITE_SIZE counter passes of "
                    "--profile-run under DIR (DIR/FETCH_SIZE/*.csv, "
                    "DIR/WRITE_SIZE/*.csv) into profiles/fobf_c3_hbm_traffic.json, then exit")
    ap.add_argument("--write-sq-summary", nargs=2, metavar=("PASS1_DIR", "PASS2_DIR"),
                    help="turn the two SQ counter passes of --profile-run (rocprofv3 "
                    "--pmc output directories) into profiles/fobf_c3_sq_counters.md, then exit")
    ap.add_argument("--write-batch-trace-summary", nargs=2, metavar=("STATS_CSV", "BENCH_JSON"),
                    help="turn a rocprofv3 --kernel-trace --stats summary of a "
                    "bench run with the batch leg (and that run's JSON line) into "
                    "profiles/fobf_c4_batch_trace.md, then exit")
    ap.add_argument("--write-serve-trace-summary", nargs=2, metavar=("TRACE_CSV", "BENCH_JSON"),
                    help="turn a rocprofv3 --kernel-trace of a bench run with the "
                    "serving leg (and that run's JSON line) into "
                    "profiles/fobf_c5_serve_trace.md, then exit")
    ap.add_argument("--write-trace-summary", nargs=2, metavar=("STATS_CSV", "BENCH_JSON"),
                    help="turn a rocprofv3 --kernel-trace --stats summary of a "
                    "bench run (and that run's JSON line) into "
                    "profiles/fobf_c3_kernel_trace.md, then exit")
    return ap.parse_args()


KERNEL_LABELS = {
    "mfma_f32_kernel_c3": "fp32 (16x16x4 f32 matrix instruction, 19 horizontal steps = r 30)",
    "mfma_f32_ws_kernel_c3": "fp32, workspace form (channels staged per workgroup, 512-row tiles)",
    "mfma_staged_f16_c3": "fp16-staged (16x16x32 f16, fp32 accumulation)",
    "mfma_staged_bf16_c3": "bf16 hi+lo staged (16x16x32 bf16, fp32 accumulation)",
    "mfma_staged_f16x2_c3": "fp16 hi+lo staged (16x16x32 f16, fp32 accumulation)",
    "mfma_staged_ws_f16_c3": "fp16-staged, workspace form (512-row tiles)",
    "mfma_staged_ws_bf16_c3": "bf16 hi+lo staged, workspace form (512-row tiles)",
    "mfma_staged_ws_f16x2_c3": "fp16 hi+lo staged, workspace form (512-row tiles)",
    "valu_kernel_c3": "fp32 vector-ALU direct FIR (comparison path, no matrix cores)",
}

# peak (TFLOP/s) each traced kernel's products run on
KERNEL_PEAK = {"mfma_f32_kernel_c3": 157.3, "mfma_f32_ws_kernel_c3": 157.3,
               "valu_kernel_c3": 157.3}


MODE_TRAFFIC = {"fp32": "mfma_f32_kernel_c3", "fp32_ws": "mfma_f32_ws_kernel_c3",
                "fp32_valu": "valu_kernel_c3",
                "fp16": "mfma_staged_f16_c3", "fp16_ws": "mfma_staged_ws_f16_c3", "bf16": "mfma_staged_bf16_c3",
                "fp16x2": "mfma_staged_f16x2_c3", "bf16_ws": "mfma_staged_ws_bf16_c3",
                "fp16x2_ws": "mfma_staged_ws_f16x2_c3"}


def mode_call(m, H, W, theta, torch):
    """(precision, workspace tensor or None, algorithm) of a bench mode name:
    a _ws suffix calls fobf_filter_ws with a workspace, fp32_valu the
    vector-ALU kernel, anything else fobf_filter on the matrix cores."""
    import paper_1811_02168_amd as F
    if m == "fp32_valu":
        return "fp32", None, "valu"
    if not m.endswith("_ws"):
        return m, None, "mfma"
    prec = m[:-3]
    n = F.filter_workspace_size(H, W, theta, prec)
    return prec, torch.empty(max(n, 1), dtype=torch.uint8, device="cuda"), "auto"


# peak of the matrix instruction each mode's products run on (dense
# MI355X figures): fp32 16x16x4 (= the fp32 vector peak), fp16 and bf16
# 16x16x32; the vector-ALU kernel against the fp32 vector peak
MODE_PEAK_TFLOPS = {"fp32": 157.3, "fp32_ws": 157.3, "fp32_valu": 157.3,
                    "fp16": 2500.0, "fp16_ws": 2500.0, "bf16": 2500.0, "bf16_ws": 2500.0,
                    "fp16x2": 2500.0, "fp16x2_ws": 2500.0}


def write_trace_summary(stats_csv, bench_json):
    """profiles/fobf_c3_kernel_trace.md from `rocprofv3 --kernel-trace --stats`
    of `bench.py --no-cpu-baseline --no-serve --no-batch`: per filter kernel,
    calls and durations, and the flop rate they imply."""
    import csv
    line = json.loads(open(bench_json).read().strip().splitlines()[-1])
    flop = line["roofline"]["flop_per_px"] * line["config"]["H"] * line["config"]["W"]
    rows = list(csv.DictReader(open(stats_csv)))
    # per-dispatch durations, in dispatch order, from the trace beside the
    # stats: the last steps x images launches of each kernel are the
    # bench's timed region (the others are its warm-up and tuning runs)
    durs = {}
    trace_csv = os.path.join(os.path.dirname(stats_csv), "fobf_kernel_trace.csv")
    if os.path.exists(trace_csv):
        for t in sorted(csv.DictReader(open(trace_csv)), key=lambda t: int(t["Dispatch_Id"])):
            durs.setdefault(t["Kernel_Name"], []).append(
                int(t["End_Timestamp"]) - int(t["Start_Timestamp"]))
    n_timed = line["steps"] * line["config"]["images_per_step"]
    out = ["# Kernel trace: 4096^2 image, theta = 10 (61 taps), K = 8, "
           "sigma in {20, 50, 100}", "",
           "Command (from the repository root on the MI355X host; "
           "`cd /tmp && export TMPDIR=/tmp` first):", "",
           "    rocprofv3 --kernel-trace --stats -d <out>/trace -o fobf "
           "--output-format csv -- \\",
           f"        python3 bench.py --steps {line['steps']} --warmup {line['warmup']} "
           "--no-cpu-baseline --no-serve --no-batch", "",
           "Summary written by `python3 bench.py --write-trace-summary "
           "<out>/trace/fobf_kernel_stats.csv <bench JSON line>`.", "",
           f"Per kernel: the average over the last {n_timed} calls, the bench's timed "
           f"region ({line['steps']} steps x {line['config']['images_per_step']} images), "
           "which the rate and fraction use; then rocprofv3's statistics over all "
           "calls (the warm-up and tuning runs included, slower first calls among "
           "them).", "",
           "| Kernel | timed-region average ns | TFLOP/s (7076 flop/px) "
           "| peak of its products (TFLOP/s) | fraction of that peak | Calls "
           "| all-calls average ns | Min ns | Max ns |",
           "|---|---|---|---|---|---|---|---|---|"]
    for key, subs in TRAFFIC_KERNELS.items():
        for r in rows:
            if any(x in r["Name"] for x in subs):
                avg = float(r["AverageNs"])
                d = durs.get(r["Name"], [])[-n_timed:]
                tavg = sum(d) / len(d) if d else avg
                tf = flop / (tavg * 1e-9) / 1e12
                pk = KERNEL_PEAK.get(key, 2500.0)
                out.append(f"| `{r['Name'][:90]}` {KERNEL_LABELS[key]} | {tavg:,.0f} | "
                           f"{tf:.1f} | {pk:g} | {tf / pk:.3f} | {r['Calls']} | "
                           f"{avg:,.0f} | {int(float(r['MinNs'])):,} | "
                           f"{int(float(r['MaxNs'])):,} |")
    out += ["", f"The traced run's own step: {line['ms_per_step']} ms for "
            f"{line['config']['images_per_step']} images (driver-side wall clock of the "
            "timed steps).", "",
            "HIP-event timing inside the same traced run (`roofline.kernel_ms` "
            f"of its JSON line): headline fp32 {line['roofline']['kernel_ms']} ms per launch; "
            + ", ".join(f"{k} {v['kernel_ms']} ms" for k, v in line.get("mixed", {}).items())
            + ".", ""]
    with open(os.path.join(ROOT, "profiles", "fobf_c3_kernel_trace.md"), "w") as fh:
        fh.write("\n".join(out))


def write_batch_trace_summary(stats_csv, bench_json):
    """profiles/fobf_c4_batch_trace.md from `rocprofv3 --kernel-trace --stats`
    of a bench run with the batch leg: the persistent batch kernels' device
    time per launch beside the bench's wall-clock time per batch."""
    import csv
    line = json.loads(open(bench_json).read().strip().splitlines()[-1])
    b = line["batch"]
    rows = list(csv.DictReader(open(stats_csv)))
    batch = [r for r in rows if "batch_kernel" in r["Name"]]
    # per-dispatch durations in dispatch order: launches 2..6 of each batch
    # kernel are the bench's 5 timed batches (the first is its untimed run)
    durs = {}
    trace_csv = os.path.join(os.path.dirname(stats_csv),
                             os.path.basename(stats_csv).replace("kernel_stats", "kernel_trace"))
    if os.path.exists(trace_csv):
        for t in sorted(csv.DictReader(open(trace_csv)), key=lambda t: int(t["Dispatch_Id"])):
            if "batch_kernel" in t["Kernel_Name"]:
                durs.setdefault(t["Kernel_Name"], []).append(
                    int(t["End_Timestamp"]) - int(t["Start_Timestamp"]))
    out = ["# Kernel trace of the batch leg: 256 uneven images (C4), 168 Mpix", "",
           "Command (from the repository root on the MI355X host; "
           "`cd /tmp && export TMPDIR=/tmp` first):", "",
           "    rocprofv3 --kernel-trace --stats -d <out>/c4 -o c4 --output-format csv -- \\",
           "        python3 bench.py --steps 1 --warmup 1 --no-cpu-baseline --no-serve "
           "--no-mixed", "",
           "Summary written by `python3 bench.py --write-batch-trace-summary "
           "<out>/c4/c4_kernel_stats.csv <bench JSON line>`.", "",
           "The persistent batch launches one kernel per precision and radius class "
           "(all of C4 is in the r <= 24 class); float32 runs 7 times (one untimed, "
           "5 timed, one for the equality check), two-word fp16 6 times.", "",
           "| Kernel | timed launches (2..6) average ns | Calls | all-calls average ns "
           "| Min ns | Max ns |",
           "|---|---|---|---|---|---|"]
    for r in batch:
        d = durs.get(r["Name"], [])[1:6]
        tavg = f"{sum(d) / len(d):,.0f}" if d else "-"
        out.append(f"| `{r['Name'][:110]}` | {tavg} | {r['Calls']} | "
                   f"{float(r['AverageNs']):,.0f} | "
                   f"{int(float(r['MinNs'])):,} | {int(float(r['MaxNs'])):,} |")
    out += ["",
            "The same run's bench line (wall clock per batch, host work included): "
            f"persistent float32 {b['persistent']['ms']} ms, two-word fp16 "
            f"{b['persistent_fp16x2']['ms']} ms, one launch per image "
            f"{b['per_image']['ms']} ms; every float32 batch image equal to its "
            f"single launch (max |difference| {b['max_abs_batch_vs_single']}).", ""]
    with open(os.path.join(ROOT, "profiles", "fobf_c4_batch_trace.md"), "w") as fh:
        fh.write("\n".join(out))


def write_serve_trace_summary(trace_csv, bench_json):
    """profiles/fobf_c5_serve_trace.md from `rocprofv3 --kernel-trace` of a
    bench run with the serving leg only: the device time of the kernels the
    server launched (from its first batch on), per kernel family, beside the
    requests' end-to-end latencies of the same run."""
    import csv
    line = json.loads(open(bench_json).read().strip().splitlines()[-1])
    sv = line["serving"]
    ds = sorted(csv.DictReader(open(trace_csv)), key=lambda t: int(t["Dispatch_Id"]))
    first = next((i for i, t in enumerate(ds) if "batch_kernel" in t["Kernel_Name"]), len(ds))
    fam = {}
    for t in ds[first:]:
        n = t["Kernel_Name"]
        key = ("persistent batch kernel" if "batch_kernel" in n else
               "workspace form (tall requests)" if "_ws_kernel" in n else
               "batch counter reset" if "reset_counter" in n else
               "HIP runtime copy kernel (host-device copies it runs as a kernel)"
               if "copyBuffer" in n else "other")
        fam.setdefault(key, []).append((int(t["End_Timestamp"]) - int(t["Start_Timestamp"])) / 1e6)

    def pct(v, q):
        v = sorted(v)
        return v[min(len(v) - 1, int(q * len(v)))]

    out = ["# Kernel trace of the serving leg (C5: Poisson arrivals at 200 requests/s, "
           "128^2..4096^2, half fp32 and half fp16-staged)", "",
           "Command (from the repository root on the MI355X host; "
           "`cd /tmp && export TMPDIR=/tmp` first):", "",
           "    rocprofv3 --kernel-trace -d <out>/c5 -o c5 --output-format csv -- \\",
           "        python3 bench.py --steps 1 --warmup 1 --no-cpu-baseline --no-batch "
           "--no-mixed --serve-requests 1000", "",
           "Summary written by `python3 bench.py --write-serve-trace-summary "
           "<out>/c5/c5_kernel_trace.csv <bench JSON line>`.", "",
           "Device time of every kernel the server launched (warm and cold legs "
           "together), per kernel family:", "",
           "| Kernel family | launches | total ms | mean ms | p50 ms | p99 ms | max ms |",
           "|---|---|---|---|---|---|---|"]
    for k, v in sorted(fam.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"| {k} | {len(v)} | {sum(v):.1f} | {sum(v) / len(v):.4f} | "
                   f"{pct(v, 0.5):.4f} | {pct(v, 0.99):.4f} | {max(v):.4f} |")
    w, c = sv["warm"], sv["cold"]
    out += ["", "The same run's requests, end to end (submit to completion, PCIe copies "
            f"included): warm cache p50 {w['p50_ms']} ms, p99 {w['p99_ms']} ms "
            f"({w['requests']} timed); cold cache p50 {c['p50_ms']} ms, p99 {c['p99_ms']} ms "
            f"({c['requests']}). Their device share (copy in, kernels, copy out) "
            f"p50 {w['breakdown_ms']['device']['p50']} / p99 "
            f"{w['breakdown_ms']['device']['p99']} ms (warm).", ""]
    with open(os.path.join(ROOT, "profiles", "fobf_c5_serve_trace.md"), "w") as fh:
        fh.write("\n".join(out))


SQ_PASSES = (
    "SQ_WAVES SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_INSTS_VALU SQ_INSTS_MFMA SQ_INSTS_LDS "
    "SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS GRBM_GUI_ACTIVE",
    "SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_WAIT_INST_LDS SQ_LDS_BANK_CONFLICT SQ_ACTIVE_INST_ANY "
    "SQ_INSTS_SALU SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_VMEM_RD",
)


def write_sq_summary(d1, d2):
    """profiles/fobf_c3_sq_counters.md from the two SQ counter passes of
    `bench.py --profile-run`: per kernel, the counter totals of its dispatch
    and the ratios that read them."""
    import csv
    import glob

    vals = {}
    for d in (d1, d2):
        files = glob.glob(os.path.join(d, "*counter_collection.csv"))
        if not files:
            raise SystemExit(f"no counter CSV under {d}")
        for r in csv.DictReader(open(files[0])):
            for key, subs in TRAFFIC_KERNELS.items():
                if any(x in r["Kernel_Name"] for x in subs):
                    e = vals.setdefault(key, {})
                    e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    keys = [k for k in TRAFFIC_KERNELS if k in vals]
    counters = " ".join(SQ_PASSES).split()
    out = ["# SQ counters of the single-image kernels (4096², θ = 10, K = 8, σ = 50)", "",
           "One launch of each kernel (the `--profile-run` leg of `bench.py`: the 4096² "
           "image, σ = 50, K = 8, fitted T), two counter passes of rocprofv3 on one MI355X "
           "(gfx950), from the repository root:", "", "```", "cd /tmp && export TMPDIR=/tmp"]
    for i, cs in enumerate(SQ_PASSES, 1):
        out.append(f"timeout -s KILL 120 rocprofv3 --pmc {cs} -d <out>/sq{i} -o p{i} "
                   "--output-format csv -- python3 bench.py --profile-run")
    out += ["python3 bench.py --write-sq-summary <out>/sq1 <out>/sq2", "```", "",
            "Values are the counter totals of the dispatch as rocprofv3 reports them "
            "(summed over the chip; cycle counters in the SQ's own units).", "",
            "| counter | " + " | ".join(KERNEL_LABELS[k].split(" (")[0] for k in keys) + " |",
            "|---|" + "---|" * len(keys)]
    for c in counters:
        out.append(f"| {c} | " + " | ".join(f"{vals[k].get(c, float('nan')):,.0f}"
                                            for k in keys) + " |")

    def ratio(num, den):
        return [vals[k].get(num, 0.0) / vals[k][den] if vals[k].get(den) else float("nan")
                for k in keys]
    rows = [("wait / wave cycles", ratio("SQ_WAIT_ANY", "SQ_WAVE_CYCLES")),
            ("waiting to issue / wave cycles", ratio("SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES")),
            ("VALU active / wave cycles", ratio("SQ_ACTIVE_INST_VALU", "SQ_WAVE_CYCLES")),
            ("LDS bank conflict / LDS active", ratio("SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_LDS")),
            ("LDS bank conflict / LDS instructions", ratio("SQ_LDS_BANK_CONFLICT", "SQ_INSTS_LDS")),
            ("VALU insts / MFMA insts", ratio("SQ_INSTS_VALU", "SQ_INSTS_MFMA"))]
    for name, v in rows:
        out.append(f"| {name} | " + " | ".join(f"{x:.2f}" for x in v) + " |")
    out += ["", f"Kernel source hash (bench.py `kernel_source_hash`): {kernel_source_hash()}.", ""]
    with open(os.path.join(ROOT, "profiles", "fobf_c3_sq_counters.md"), "w") as fh:
        fh.write("\n".join(out))


def profile_run(modes):
    import numpy as np
    import torch

    import paper_1811_02168_amd as F
    import workloads

    cfg = workloads.C3
    dev = torch.device("cuda")
    a = torch.ones(64 << 20, dtype=torch.float32, device=dev)     # 256 MiB
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    img = torch.from_numpy(cfg.image().astype(np.float32)).to(dev)
    out = torch.empty_like(img)
    coef = F.fit(cfg.R, 50.0, cfg.K, eps=cfg.eps)
    for m in modes:
        prec, ws, algo = mode_call(m, cfg.H, cfg.W, cfg.theta, torch)
        F.filter(img, cfg.theta, cfg.K, coef.T, coef.c, prec=prec, algo=algo, out=out,
                 workspace=ws)
        torch.cuda.synchronize()
        print(f"[profile-run] {m} done", file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the device code and its launch configuration (kernel bodies,
    launchers, tile-height defaults) with comments and blank space removed,
    so that only code changes invalidate recorded counters."""
    import re
    h = hashlib.sha256()
    for name in ("fobf_tiles.h", "fobf_mfma.hip", "fobf_mfma_ws.hip", "fobf_tune.hip",
                 "fobf_valu.hip"):
        with open(os.path.join(ROOT, "paper_1811_02168_amd", "csrc", name)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


TRAFFIC_KERNELS = {            # key -> substrings naming the kernel
    "mfma_f32_kernel_c3": ("mfma_f32_kernel<19>", "mfma_f32_kernelILi19E"),
    "mfma_f32_ws_kernel_c3": ("mfma_f32_ws_kernel<19>", "mfma_f32_ws_kernelILi19E"),
    "mfma_staged_f16_c3": ("mfma_staged_kernel<_Float16, 5>", "mfma_staged_kernelIDF16_Li5E"),
    "mfma_staged_bf16_c3": ("mfma_staged_kernel<__bf16, 5>", "mfma_staged_kernelIDF16bLi5E"),
    "mfma_staged_f16x2_c3": ("mfma_staged_kernel<fobf::(anonymous namespace)::F16Pair, 5>",
                             "mfma_staged_kernelINS0_7F16PairELi5E"),
    "mfma_staged_ws_f16_c3": ("mfma_staged_ws_kernel<_Float16, 5>",
                              "mfma_staged_ws_kernelIDF16_Li5E"),
    "mfma_staged_ws_bf16_c3": ("mfma_staged_ws_kernel<__bf16, 5>",
                               "mfma_staged_ws_kernelIDF16bLi5E"),
    "mfma_staged_ws_f16x2_c3": ("mfma_staged_ws_kernel<fobf::(anonymous namespace)::F16Pair, 5>",
                                "mfma_staged_ws_kernelINS0_7F16PairELi5E"),
    "valu_kernel_c3": ("valu_kernel(", "valu_kernelENS_11ImageParamsE"),
}


def write_traffic(d):
    """profiles/fobf_c3_hbm_traffic.json from two rocprofv3 --pmc passes of
    `bench.py --profile-run`: per kernel, FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch) scaled by the factor that makes each counter read 256 MiB for
    the 256 MiB device-to-device copy of the same run."""
    import csv
    import glob

    def rows(counter):
        files = glob.glob(os.path.join(d, counter, "*counter_collection.csv"))
        if not files:
            raise SystemExit(f"no {counter} counter CSV under {d}")
        per = {}
        for r in csv.DictReader(open(files[0])):
            if r["Counter_Name"] != counter:
                continue
            key = (r["Dispatch_Id"], r["Kernel_Name"])
            per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
        return per

    fetch, write = rows("FETCH_SIZE"), rows("WRITE_SIZE")
    copy_kib = 256 * 1024.0

    def copy_read(per):
        vals = [v for (_, name), v in per.items() if "copyBuffer" in name]
        if not vals:
            raise SystemExit("the calibration copy is missing from the counter pass")
        return max(vals)

    fr, wr = copy_read(fetch), copy_read(write)
    fs, ws = copy_kib / fr, copy_kib / wr
    alg = 8 * 4096 * 4096
    out = {
        "_comment": "HBM traffic per launch of the 4096^2, theta=10, K=8, sigma=50 "
        "filter. FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two rocprofv3 "
        "--pmc runs of `python3 bench.py --profile-run`, each scaled by the factor "
        "that makes the same counter read 256 MiB for the 256 MiB device copy in "
        "that run; written by `python3 bench.py --write-traffic <out>`. source_hash "
        "identifies the kernel sources the counters were taken from; bench.py "
        "reports traffic only while it matches.",
        "commands": [
            "rocprofv3 --pmc FETCH_SIZE -d <out>/FETCH_SIZE -o FETCH_SIZE "
            "--output-format csv -- python3 bench.py --profile-run",
            "rocprofv3 --pmc WRITE_SIZE -d <out>/WRITE_SIZE -o WRITE_SIZE "
            "--output-format csv -- python3 bench.py --profile-run",
            "python3 bench.py --write-traffic <out>",
        ],
        "copy_calibration": {"fetch_kib_read": fr, "write_kib_read": wr,
                             "fetch_scale": fs, "write_scale": ws},
    }
    for key, subs in TRAFFIC_KERNELS.items():
        f = [(n, v) for (_, n), v in fetch.items() if any(x in n for x in subs)]
        w = [(n, v) for (_, n), v in write.items() if any(x in n for x in subs)]
        if not f or not w:
            continue
        fk, wk = f[0][1], w[0][1]
        b = int(round((fk * fs + wk * ws) * 1024))
        out[key] = {"kernel": f[0][0], "source_hash": kernel_source_hash(),
                    "fetch_kib": fk, "write_kib": wk, "bytes_per_launch": b,
                    "algorithmic_bytes": alg, "ratio_to_algorithmic": round(b / alg, 4)}
    with open(os.path.join(ROOT, "profiles", "fobf_c3_hbm_traffic.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps({k: v.get("ratio_to_algorithmic") for k, v in out.items()
                      if isinstance(v, dict) and "ratio_to_algorithmic" in v}))


def traffic_record(kernel_key, launches_bytes_alg):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when that summary is missing or was taken from other kernel code."""
    path = os.path.join(ROOT, "profiles", "fobf_c3_hbm_traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = rec.get(kernel_key)
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def main():
    args = parse()
    if args.write_traffic:
        write_traffic(args.write_traffic)
        return
    if args.write_trace_summary:
        write_trace_summary(*args.write_trace_summary)
        return
    if args.write_batch_trace_summary:
        write_batch_trace_summary(*args.write_batch_trace_summary)
        return
    if args.write_serve_trace_summary:
        write_serve_trace_summary(*args.write_serve_trace_summary)
        return
    if args.write_sq_summary:
        write_sq_summary(*args.write_sq_summary)
        return
    if args.profile_run:
        profile_run([m for m in args.modes.split(",") if m])
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; "
                          f"--gpus {args.gpus} is not supported"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1811_02168_amd as F
    import workloads

    cfg = workloads.C3
    theta, K, R = cfg.theta, cfg.K, cfg.R
    r = math.ceil(3 * theta)
    flop_px = 4 * (2 * r + 1) * (4 * K - 3)
    H, W = cfg.H, cfg.W
    npx = H * W
    f = cfg.image()
    cpu, refs = None, None
    if not args.no_cpu_baseline:
        cpu, refs = cpu_baseline_leg(f, cfg)
        print(f"[bench] cpu baseline: {cpu}", file=sys.stderr, flush=True)
    dev = torch.device("cuda")
    img = torch.from_numpy(f.astype(np.float32)).to(dev)
    outs = {s: torch.empty_like(img) for s in cfg.sigmas}
    stream = torch.cuda.current_stream()

    calls = {}

    def step(mode):
        if mode not in calls:
            calls[mode] = mode_call(mode, H, W, theta, torch)
        prec, ws, algo = calls[mode]
        for s in cfg.sigmas:
            coef = F.fit(R, s, K, eps=cfg.eps)         # cached host fit
            F.filter(img, theta, K, coef.T, coef.c, prec=prec, algo=algo, out=outs[s],
                     workspace=ws)

    def timed(prec, steps, warmup):
        for _ in range(warmup):
            step(prec)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t0 = time.perf_counter()
        for i in range(steps):
            ev[i][0].record(stream)
            step(prec)
            ev[i][1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gpu_ms = sum(a.elapsed_time(b) for a, b in ev) / steps
        ms_step = wall * 1e3 / steps
        nimg = len(cfg.sigmas)
        return {
            "ms_per_step": ms_step,
            "kernel_ms": gpu_ms / nimg,          # average per launch
            "value": nimg * npx / (ms_step * 1e-3) / 1e6,
        }

    # a1, the host fit: cold cost of the period scan per (sigma, K), of
    # Algorithm 1, and of one read-out of a (sigma, eps) table
    F.fit_cache_clear()
    host_fit = {}
    for s in cfg.sigmas:
        t0 = time.perf_counter()
        F.fit(R, s, K, eps=cfg.eps)                    # cached for the steps
        host_fit[f"scan_K{K}_sigma{s:g}_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    t0 = time.perf_counter()
    a1 = F.fit(R, 50.0, 0, eps=1e-3)
    host_fit["algorithm1_sigma50_eps1e-3_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    host_fit["algorithm1_K"] = a1.K
    lut = F.Lut.create(R, [20.0, 40.0, 80.0], [1e-1, 1e-3])
    t0 = time.perf_counter()
    for _ in range(100):
        lut.fit(33.0, 1e-2)
    host_fit["table_readout_us"] = round((time.perf_counter() - t0) * 1e4, 1)
    lut.close()
    modes = [m for m in args.modes.split(",") if m]
    if args.no_mixed:
        modes = ["fp32_ws"]
    # untimed device warm-up (~0.1 s of the plain fp32 kernel): the first
    # launches after idle run at lower clocks (measured: 1.75 -> 1.49 ms over
    # the first 20 launches of a kernel started cold)
    for _ in range(20):
        F.filter(img, theta, K, F.fit(R, 50.0, K, eps=cfg.eps).T,
                 F.fit(R, 50.0, K, eps=cfg.eps).c, prec="fp32", out=outs[cfg.sigmas[0]])
    torch.cuda.synchronize()
    res = {}
    for m in modes:
        res[m] = timed(m, args.steps, args.warmup)
        print(f"[bench] {m}: {res[m]}", file=sys.stderr, flush=True)

    # the headline: float32, through fobf_filter_ws when that mode ran (its
    # output equals fobf_filter's bit for bit), else through fobf_filter
    head = "fp32_ws" if "fp32_ws" in res else "fp32"
    main_res = res[head]
    achieved = flop_px * npx / (main_res["kernel_ms"] * 1e-3) / 1e12
    alg_bytes = 8 * npx
    traffic = traffic_record(MODE_TRAFFIC[head], alg_bytes)
    roofline = {
        "bound": "mfma",
        "achieved": round(achieved, 2),
        "peak": PEAK_FP32_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
        "traffic": traffic,
        "kernel": ("mfma_f32_ws_kernel<SH=19> (fobf_filter_ws)" if head == "fp32_ws"
                   else "mfma_f32_kernel<SH=19> (fobf_filter)"),
        "kernel_ms": round(main_res["kernel_ms"], 4),
        "flop_per_px": flop_px,
        "hbm_gbs_algorithmic": round(alg_bytes / (main_res["kernel_ms"] * 1e-3) / 1e9, 1),
    }

    # measured ceilings of the instruction classes the kernels use
    measured = {}
    for kind in F.fobf.PEAK_KINDS:
        try:
            measured[kind] = round(F.peak(kind), 2)
        except Exception as e:  # reported, never hidden
            measured[kind] = repr(e)
    roofline["measured_peak_tflops"] = measured
    if isinstance(measured.get("mfma_f32"), float):
        roofline["frac_of_measured_mfma_f32"] = round(achieved / measured["mfma_f32"], 4)
    # the vector-ALU FMA rate code built without packed fp32 can issue
    if isinstance(measured.get("valu_fma_f32"), float):
        roofline["frac_of_measured_valu_fma_f32"] = round(achieved / measured["valu_fma_f32"], 4)
    print(f"[bench] measured peaks: {measured}", file=sys.stderr, flush=True)

    # the other modes: each against the peak of the matrix instruction its
    # products run on (fp16 / bf16: 2.5 PFLOP/s dense), with the HBM bytes
    # one launch moves (rocprofv3 counters, while they match the code)
    mixed = {}
    for m in modes:
        if m == head:
            continue
        a = flop_px * npx / (res[m]["kernel_ms"] * 1e-3) / 1e12
        hb = traffic_record(MODE_TRAFFIC.get(m, ""), alg_bytes)
        name = {"fp32": "fp32_fobf_filter", "fp32_valu": "fp32_valu"}.get(m, m + "_stage")
        mixed[name] = {
            "value": round(res[m]["value"], 1), "unit": "Mpix/s",
            "ms_per_step": round(res[m]["ms_per_step"], 4),
            "kernel_ms": round(res[m]["kernel_ms"], 4),
            "tflops_equiv": round(a, 2),
            "peak_tflops": MODE_PEAK_TFLOPS[m],
            "frac_of_peak": round(a / MODE_PEAK_TFLOPS[m], 4),
            "hbm_bytes_per_launch": hb,
            "hbm_tbs": round(hb / (res[m]["kernel_ms"] * 1e-3) / 1e12, 3) if hb else None}

    accuracy = None
    if not args.no_cpu_baseline:
        accuracy = accuracy_leg(img, cfg, modes, refs, F, torch)
        refs = None

    small = None
    if not args.no_mixed:
        try:
            small = small_configs_leg(F, torch)
        except Exception as e:  # reported, never hidden
            small = {"error": repr(e)}
        print(f"[bench] small configs: {small}", file=sys.stderr, flush=True)

    batch = None
    if not args.no_batch:
        try:
            batch = batch_leg(F, torch, args.batch_images)
        except Exception as e:  # reported, never hidden
            batch = {"error": repr(e)}
        print(f"[bench] batch: {batch}", file=sys.stderr, flush=True)

    serving = None
    if not args.no_serve:
        try:
            from paper_1811_02168_amd import serving as S
            serving = {"warm": S.bench_serving(f, n=args.serve_requests,
                                               warmup=args.serve_requests // 10),
                       "cold": S.bench_serving(f, n=args.serve_requests // 4,
                                               warmup=0, warm_cache=False,
                                               seed=2005)}
        except Exception as e:  # reported, never hidden
            serving = {"error": repr(e)}

    line = {
        "metric": "Mpix/s FOBF K=8 theta=10 4096^2 (fp32 plain; mixed below)",
        "value": round(main_res["value"], 1),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "C3: 4096x4096 Voronoi+ramp+noise, theta=10 "
                   "(61 taps), K=8, R=255, sigma in {20,50,100}; one step = "
                   "3 filtered images", "images_per_step": len(cfg.sigmas),
                   "H": H, "W": W, "theta": theta, "K": K,
                   "sigmas": list(cfg.sigmas),
                   "entry_point": ("fobf_filter_ws (float32 workspace form; output "
                                   "identical to fobf_filter)" if head == "fp32_ws"
                                   else "fobf_filter")},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "mixed": mixed,
        "accuracy_vs_fp64_oracle": accuracy,
        "host_fit": host_fit,
        "small_configs": small,
        "batch": batch,
        "serving": serving,
    }
    print(json.dumps(line))


def small_configs_leg(F, torch):
    """The two smaller parity workloads (256^2, theta = 3, K = 4; 1024^2,
    theta = 5, K = 6) through fobf_filter, fp32 and fp16 staging, resident
    inputs: per-image kernel time by HIP events over repeated launches on
    the current stream (context beside the paper's 256^2 timings)."""
    import workloads
    out = {}
    st = torch.cuda.current_stream()
    for cfg in (workloads.C1, workloads.C2):
        img = torch.from_numpy(cfg.image().astype("float32")).cuda()
        o = torch.empty_like(img)
        rec = {"H": cfg.H, "W": cfg.W, "theta": cfg.theta, "K": cfg.K}
        for prec in ("fp32", "fp16"):
            ms = []
            for sigma in cfg.sigmas:
                co = F.fit(255, sigma, cfg.K, eps=cfg.eps)
                call = lambda: F.filter(img, cfg.theta, cfg.K, co.T, co.c, prec=prec, out=o)
                for _ in range(10):
                    call()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(st)
                for _ in range(50):
                    call()
                e1.record(st)
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1) / 50)
            avg = sum(ms) / len(ms)
            rec[prec] = {"kernel_ms": round(avg, 4),
                         "mpix_s": round(cfg.H * cfg.W / (avg * 1e-3) / 1e6, 1)}
        out[cfg.name] = rec
    return out


def batch_leg(F, torch, n):
    """C4: n uneven images (log-uniform area 64^2..2048^2, theta in [2,8],
    K in 3..10, fp32): the autotuned persistent batched launch against one
    fobf_filter launch per image, both on resident inputs.  Each image is a
    seeded window of the 4096^2 test image (same generator and statistics
    as the per-job images, without generating 168 Mpix on the host)."""
    import numpy as np

    import workloads

    pool = workloads.C3.image()
    rng = np.random.default_rng(1044)

    t0 = time.perf_counter()
    F.autotune("fp32", 2048, 2048, 6)
    tune_s = time.perf_counter() - t0
    jobs = workloads.batch_jobs(n=n)
    dev = torch.device("cuda")
    items, descs = [], []
    for j in jobs:
        y = int(rng.integers(0, pool.shape[0] - j.H + 1))
        x = int(rng.integers(0, pool.shape[1] - j.W + 1))
        win = np.ascontiguousarray(pool[y:y + j.H, x:x + j.W], dtype=np.float32)
        img = torch.from_numpy(win).to(dev)
        out = torch.empty_like(img)
        coef = F.fit(255, j.sigma, j.K, eps=0.1)
        items.append((img, out, j, coef))
        descs.append(F.make_job(img, out, j.theta, j.K, coef.T, coef.c))
    mpix = sum(j.H * j.W for j in jobs) / 1e6
    flop = sum(4 * (2 * math.ceil(3 * j.theta) + 1) * (4 * j.K - 3) * j.H * j.W
               for j in jobs)
    # matrix-core flops the fp32 batch body executes: per tile of 4 strips x
    # nblk blocks and per channel, (nblk + DV - 1) horizontal 16-row blocks
    # and nblk vertical blocks, each of SH = ceil((16 + 2r) / 4) steps, a
    # step a 16x16x4 product (2048 flop); at small radii the 16-wide band
    # of the Toeplitz products is mostly zero taps (r = 6: 28 columns and
    # 28 rows for 13 taps)
    exec_flop = 0
    for j in jobs:
        r = math.ceil(3 * j.theta)
        dv = (16 + 2 * r + 15) // 16
        sh = (16 + 2 * r + 3) // 4
        nblk = F.tune_get("fp32", j.theta)[1]
        nblk = max(1, min(nblk, 8, (j.H + 15) // 16))
        ntx, nty = -(-j.W // 64), -(-j.H // (16 * nblk))
        exec_flop += (ntx * nty * 4 * 2048 * (4 * j.K - 3) *
                      (sh * (nblk + dv - 1) + sh * nblk))
    ws = torch.empty(F.batch_workspace_size(len(descs)), dtype=torch.uint8, device=dev)

    def run_batch():
        F.filter_batch(descs, workspace=ws)

    def run_single():
        for img, out, j, coef in items:
            F.filter(img, j.theta, j.K, coef.T, coef.c, out=out)

    res = {}
    for name, fn in (("persistent", run_batch), ("per_image", run_single)):
        fn()
        torch.cuda.synchronize()
        reps = 5
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / reps
        res[name] = {"ms": round(ms, 3), "mpix_s": round(mpix / ms * 1e3, 1),
                     "tflops": round(flop / ms / 1e9, 2)}
    res["persistent"]["mfma_executed_tflops"] = round(exec_flop / res["persistent"]["ms"] / 1e9, 2)
    res["persistent"]["frac_of_peak_executed"] = round(
        exec_flop / res["persistent"]["ms"] / 1e9 / PEAK_FP32_TFLOPS, 4)
    res["executed_over_algorithmic_flop"] = round(exec_flop / flop, 3)
    # the batched results equal the per-image ones
    outs = [o.clone() for _, o, _, _ in items]
    run_batch()
    torch.cuda.synchronize()
    diff = max(float((o - b).abs().max()) for (_, o, _, _), b in zip(items, outs))
    res.update({"images": len(jobs), "mpix": round(mpix, 2),
                "speedup": round(res["per_image"]["ms"] / res["persistent"]["ms"], 3),
                "max_abs_batch_vs_single": diff, "autotune_s": round(tune_s, 2),
                "dtype": "f32"})
    # the same batch with two-word fp16 staging (float32-class accuracy)
    descs2 = [F.make_job(img, out, j.theta, j.K, coef.T, coef.c, prec="fp16x2")
              for img, out, j, coef in items]
    F.filter_batch(descs2, workspace=ws)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(5):
        F.filter_batch(descs2, workspace=ws)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / 5
    d2 = max(float((o - b).abs().max()) for (_, o, _, _), b in zip(items, outs))
    res["persistent_fp16x2"] = {"ms": round(ms, 3), "mpix_s": round(mpix / ms * 1e3, 1),
                                "tflops": round(flop / ms / 1e9, 2),
                                "max_abs_vs_fp32_per_image": d2}
    F.tune_reset()
    return res


def cpu_baseline_leg(f, cfg):
    """The bench's oracle leg, the only part of it that touches the FP64
    oracle.  It times the oracle and computes the reference values of the
    accuracy statement:

    * one core: ``fourier_direct`` (float64 numpy) on a 1024 x 1024 crop of
      the 4096^2 image at sigma = 50, best of 3 after one warm-up run;
    * every host core (up to 16 worker processes over row bands with r
      halo rows, bit-identical to one process): the whole 4096^2 image at
      each sigma, with the oracle's own fit (T, c) -- these are the
      references every GPU mode is compared with on every pixel, and the
      best of the three runs is the all-cores rate;
    * eq. (1) with the Gaussian range kernel (brute force) at 406 sampled
      pixels, for the approximation error of the K-term series (Sec. III's
      PSNR against the exact bilateral filter)."""
    import numpy as np

    import oracle as O
    from oracle.bands import BandPool, default_workers

    n = 1024
    crop = np.ascontiguousarray(f[:n, :n])
    ref50 = O.fit(cfg.R, 50.0, cfg.K)
    O.fourier_direct(crop, cfg.theta, cfg.K, ref50["T"], ref50["c"])      # warm-up
    runs = []
    for _ in range(3):
        t0 = time.perf_counter()
        O.fourier_direct(crop, cfg.theta, cfg.K, ref50["T"], ref50["c"])
        runs.append(time.perf_counter() - t0)
    dt = min(runs)
    cpu = {"value": round(n * n / dt / 1e6, 4), "unit": "Mpix/s", "cores": 1,
           "kind": "oracle",
           "sample": f"fourier_direct (float64 numpy) on the top-left {n}x{n} crop of "
                     f"the 4096^2 image, sigma=50, K={cfg.K}, theta={cfg.theta}; best of "
                     f"3 runs after one warm-up ({', '.join(f'{r:.2f}' for r in runs)} s)",
           "host_cpus": os.cpu_count()}
    rng = np.random.default_rng(77)
    H, W = f.shape
    ys = np.concatenate([rng.integers(0, H, 400), [0, 0, H - 1, H - 1, 17, H - 5]])
    xs = np.concatenate([rng.integers(0, W, 400), [0, W - 1, 0, W - 1, W - 3, 9]])
    refs = {"full": {}, "approx": {"ys": ys, "xs": xs}}
    nproc = default_workers()
    times = []
    with BandPool(nproc) as pool:
        pool.fourier_direct(crop, cfg.theta, cfg.K, ref50["T"], ref50["c"])   # warm-up
        for s in cfg.sigmas:
            fit = O.fit(cfg.R, s, cfg.K)
            t0 = time.perf_counter()
            out, num, den, Wi = pool.fourier_direct(f, cfg.theta, cfg.K, fit["T"], fit["c"])
            times.append(time.perf_counter() - t0)
            refs["full"][s] = (fit["T"], np.asarray(fit["c"], dtype=np.float64), out, den / Wi)
            del num, den, Wi
            bf, _, _ = O.brute_bf_points(f, cfg.theta, O.gaussian_range(s), ys, xs)
            refs["approx"][s] = bf
    cpu["all_cores"] = {"value": round(H * W / min(times) / 1e6, 4), "unit": "Mpix/s",
                        "cores": nproc, "seconds": [round(t, 2) for t in times],
                        "sample": "fourier_direct on the whole 4096^2 image, one run per "
                                  "sigma (the references of the accuracy statement); best "
                                  "of the 3 after a warm-up"}
    return cpu, refs


def accuracy_leg(img, cfg, modes, refs, F, torch):
    """Every precision against the FP64 oracle on every pixel of the 4096^2
    image, per sigma, with the oracle's (K, T, c): max-abs on pixels whose
    oracle denominator has D/W >= 0.01 and on the masked rest, the masked
    count, and PSNR over the whole image (Sec. III's metric) and over the
    unmasked pixels.  For float32, also the approximation error of the
    K-term series itself: the output against eq. (1) with the Gaussian
    range kernel at sampled pixels (Table I's PSNR, here at sampled
    pixels)."""
    import numpy as np

    def psnr(d):
        if d.size == 0 or not np.all(np.isfinite(d)):
            return None
        mse = float(np.mean(d * d))
        return None if mse == 0.0 else round(10 * math.log10(255.0 ** 2 / mse), 2)

    out = torch.empty_like(img)
    acc = {}
    ys, xs = refs["approx"]["ys"], refs["approx"]["xs"]
    for m in modes:
        per = {}
        for s in cfg.sigmas:
            T, c, ref, dw = refs["full"][s]
            prec, ws, algo = mode_call(m, cfg.H, cfg.W, cfg.theta, torch)
            F.filter(img, cfg.theta, cfg.K, T, c, prec=prec, algo=algo, out=out, workspace=ws)
            torch.cuda.synchronize()
            got = out.cpu().numpy().astype(np.float64)
            d = got - ref
            mask = dw >= 0.01
            masked = int(mask.size - np.count_nonzero(mask))
            e = {"maxabs_unmasked": float(np.max(np.abs(d[mask]))),
                 "masked": masked,
                 "maxabs_masked": float(np.max(np.abs(d[~mask]))) if masked else 0.0,
                 "psnr_db": psnr(d), "psnr_unmasked_db": psnr(d[mask]),
                 "min_dw": round(float(dw.min()), 4),
                 "prec_used": F.effective_prec(prec, cfg.K, T, c)}
            if m in ("fp32", "fp32_ws"):
                a = got[ys, xs] - refs["approx"][s]
                e["approx_vs_eq1_gaussian"] = {"maxabs": float(np.max(np.abs(a))),
                                               "psnr_db": psnr(a), "pixels": len(a)}
            per[f"sigma{s:g}"] = e
            del got, d
        acc[m] = {"pixels_per_sigma": cfg.H * cfg.W,
                  "maxabs_unmasked": max(v["maxabs_unmasked"] for v in per.values()),
                  "masked": sum(v["masked"] for v in per.values()),
                  "per_sigma": per}
    return acc


if __name__ == "__main__":
    main()
