"""Build libfobf.so (HIP for gfx950 + host C++) in-tree with hipcc, and
its debug-check twin libfobf_check.so (FOBF_CHECKS=1).

Usage: python paper_1811_02168_amd/build.py [release|check ...]
(or call build()).  Every call recompiles all sources of each target.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libfobf.so")
CHECK_LIB = os.path.join(HERE, "libfobf_check.so")
BUILD_CHECK = os.path.join(HERE, "_build_check")

SOURCES = [
    "fobf_api.cpp",
    "fobf_fit.cpp",
    "fobf_lut.cpp",
    "fobf_valu.hip",
    "fobf_mfma.hip",
    "fobf_mfma_ws.hip",
    "fobf_static.hip",
    "fobf_batch.hip",
    "fobf_batch_staged.hip",
    "fobf_tune.hip",
    "fobf_serve.cpp",
    "fobf_peak.hip",
    "fobf_check.cpp",
]

ARCH = "gfx950"


def hipcc() -> str:
    env = os.environ.get("HIPCC")
    if env:
        return env
    for cand in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (set HIPCC)")


def common_flags() -> list:
    return [
        "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
        # packed fp32 VALU ops stay disabled in every device code object
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", INCLUDE, "-Wall", "-Wno-unused-function",
        "-Wno-unused-command-line-argument",
    ]


def _compile(job) -> str:
    src, outdir, defs = job
    obj = os.path.join(outdir, os.path.basename(src) + ".o")
    cmd = [hipcc()] + common_flags() + list(defs)
    if src.endswith(".hip"):
        cmd += ["-x", "hip"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def _link(objs, lib: str) -> None:
    tmp = lib + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + [
        "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)


# (library, object folder, extra flags): the release library, and the
# debug-check build of the same sources (LDS poisoning and index checks,
# violations reported through fobf_check_take)
TARGETS = {
    "release": (LIB, BUILD, ()),
    "check": (CHECK_LIB, BUILD_CHECK, ("-DFOBF_CHECKS=1",)),
}


def build(verbose: bool = False, targets=("release", "check")) -> str:
    """Compile every source for each target in one pool, then link."""
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = []
    for t in targets:
        lib, outdir, defs = TARGETS[t]
        os.makedirs(outdir, exist_ok=True)
        jobs += [(s, outdir, defs) for s in srcs]
    # longest compiles first
    jobs.sort(key=lambda j: os.path.getsize(os.path.join(CSRC, j[0])), reverse=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        objs = dict(zip(jobs, ex.map(_compile, jobs)))
    for t in targets:
        lib, outdir, defs = TARGETS[t]
        _link([objs[(s, outdir, defs)] for s in srcs], lib)
        if verbose:
            print(f"built {lib}")
    return LIB


if __name__ == "__main__":
    build(verbose=True, targets=tuple(sys.argv[1:]) or ("release", "check"))
    sys.exit(0)
