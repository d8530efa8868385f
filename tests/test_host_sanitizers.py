"""The host-side C++ of the library (the float64 fit, Algorithm 1, the
fixed-period fit and the (K*, T*) table) built with AddressSanitizer and
UndefinedBehaviorSanitizer by the system g++ and driven through its C ABI
on the CPU: no out-of-bounds access, leak, use-after-free or undefined
behaviour on valid and invalid calls."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1811_02168_amd", "csrc")

DRIVER = r'''
#include <cmath>
#include <cstdio>
#include <string>
#include "fobf.h"

namespace fobf {
thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }
fobf_status fail(fobf_status st, const std::string& m) { g_err = m; return st; }
}

static int check(bool ok, const char* what) {
  if (!ok) std::printf("FAILED: %s\n", what);
  return ok ? 0 : 1;
}

int main(int argc, char** argv) {
  int bad = 0;
  fobf_coef c;
  bad += check(fobf_fit(255, 50.0, 4, 0.1, 0, &c) == FOBF_OK && c.T == 203, "fig1");
  bad += check(fobf_fit(255, 30.0, 4, 0.1, 0, &c) == FOBF_WARN_TOL, "warn");
  bad += check(fobf_fit(255, 50.0, 0, 0.1, 0, &c) == FOBF_OK && c.K == 4, "alg1");
  bad += check(fobf_fit(40, 7.0, 32, 1e-3, 0, &c) >= 0, "kmax");
  bad += check(fobf_fit(3, 2.0, 4, 0.1, 0, &c) >= 0, "K = R + 1");
  bad += check(fobf_fit(0, 50.0, 4, 0.1, 0, &c) == FOBF_EINVAL, "R = 0");
  bad += check(fobf_fit(255, NAN, 4, 0.1, 0, &c) == FOBF_EINVAL, "nan sigma");
  bad += check(fobf_fit(255, 50.0, 33, 0.1, 0, &c) == FOBF_EINVAL, "K > KMAX");
  bad += check(fobf_fit(255, 50.0, 4, 0.1, 0, nullptr) == FOBF_EINVAL, "null out");
  double b[64];
  for (int t = 0; t < 64; ++t) b[t] = 1.0 / (1.0 + t * t / 100.0);
  bad += check(fobf_fit_samples(63, b, 5, 1e9, 0, &c) == FOBF_OK, "samples");
  bad += check(fobf_fit_samples(63, nullptr, 5, 1e9, 0, &c) == FOBF_EINVAL, "null b");
  bad += check(fobf_fit_period(255, 40.0, 4, 255, &c) == FOBF_OK && c.T == 255, "period");
  bad += check(fobf_fit_period(255, 40.0, 6, 2, &c) == FOBF_EINVAL, "period rank");
  bad += check(fobf_fit_warm(255, 50.0, 4, 0.1, 0, 0, &c) == FOBF_OK && c.T == 203, "warm");
  bad += check(fobf_fit_warm(255, 50.0, 8, 0.1, 0, 2000, &c) == FOBF_OK, "warm clamp");
  bad += check(fobf_fit_warm(255, 50.0, 0, 0.1, 0, 0, &c) == FOBF_EINVAL, "warm K = 0");
  bad += check(fobf_fit_warm(255, 50.0, 4, 0.1, 0, 0, nullptr) == FOBF_EINVAL, "warm null");
  {
    const std::string cpath = std::string(argv[1]) + "/fits.txt";
    bad += check(fobf_fit_cache_save(cpath.c_str()) == FOBF_OK, "cache save");
    bad += check(fobf_fit_cache_load(cpath.c_str()) == FOBF_OK, "cache load");
    bad += check(fobf_fit_cache_load("/nonexistent/x") == FOBF_EINVAL, "cache load missing");
  }
  bad += check(fobf_fit_cache_clear() >= 1, "cache clear");
  const double sig[3] = {20.0, 40.0, 80.0}, eps[2] = {1e-1, 1e-3};
  fobf_lut* lut = nullptr;
  bad += check(fobf_lut_create(255, sig, 3, eps, 2, 0, &lut) == FOBF_OK, "lut create");
  int K = 0, T = 0;
  bad += check(fobf_lut_get(lut, 2, 1, &K, &T) == FOBF_OK && K >= 1, "lut get");
  bad += check(fobf_lut_get(lut, 3, 0, &K, &T) == FOBF_EINVAL, "lut get range");
  bad += check(fobf_lut_fit(lut, 33.0, 1e-2, &c) >= 0, "lut fit");
  bad += check(fobf_lut_fit(lut, 10.0, 1e-2, &c) == FOBF_EINVAL, "lut outside");
  const std::string path = std::string(argv[1]) + "/lut.txt";
  bad += check(fobf_lut_save(lut, path.c_str()) == FOBF_OK, "lut save");
  fobf_lut* back = nullptr;
  bad += check(fobf_lut_load(path.c_str(), &back) == FOBF_OK, "lut load");
  fobf_lut* missing = nullptr;
  bad += check(fobf_lut_load("/nonexistent/x", &missing) == FOBF_EINVAL && !missing,
               "lut load missing");
  const double bad_sig[2] = {40.0, 20.0};
  fobf_lut* none = nullptr;
  bad += check(fobf_lut_create(255, bad_sig, 2, eps, 2, 0, &none) == FOBF_EINVAL, "lut order");
  fobf_lut_destroy(lut);
  fobf_lut_destroy(back);
  fobf_lut_destroy(nullptr);
  std::printf(bad ? "failures: %d\n" : "ok\n", bad);
  return bad ? 1 : 0;
}
'''


def test_host_library_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    (tmp_path / "driver.cpp").write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "fobf_fit.cpp"), os.path.join(CSRC, "fobf_lut.cpp"),
           str(tmp_path / "driver.cpp"), "-o", str(exe), "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe), str(tmp_path)], capture_output=True, text=True,
                       env=env, timeout=600)
    if r.returncode != 0 and "LeakSanitizer does not work under ptrace" in r.stderr:
        env["ASAN_OPTIONS"] = "detect_leaks=0"
        r = subprocess.run([str(exe), str(tmp_path)], capture_output=True, text=True,
                           env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
