// C ABI entry points: validation, parameter packing and dispatch.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>

#include "fobf_internal.h"

namespace fobf {

namespace {
thread_local std::string t_error;
}

void set_error(const std::string& msg) { t_error = msg; }

fobf_status fail(fobf_status st, const std::string& msg) {
  t_error = msg;
  return st;
}

static const char* error_cstr() { return t_error.c_str(); }

int spatial_radius(double theta) {
  if (!(theta > 0.0) || !std::isfinite(theta)) return -1;
  const double r = std::ceil(3.0 * theta);
  if (r > 1e6) return -1;
  return static_cast<int>(r);
}

void make_params(ImageParams& p, const float* in, float* out, int H, int W,
                 int ld_in, int ld_out, double theta, int K, int T,
                 const double* c) {
  std::memset(&p, 0, sizeof(p));
  p.in = in;
  p.out = out;
  p.H = H;
  p.W = W;
  p.ld_in = ld_in;
  p.ld_out = ld_out;
  p.r = spatial_radius(theta);
  p.K = K;
  p.inv_period = static_cast<float>(1.0 / (2.0 * T + 1.0));
  p.check = check_word();
  for (int k = 0; k < K; ++k) p.c[k] = static_cast<float>(c[k]);
  const int r = p.r;
  double acc = 0.0;
  p.gsum[0] = 0.f;
  for (int m = -r; m <= r; ++m) {
    const double g = std::exp(-static_cast<double>(m) * m / (2.0 * theta * theta));
    if (m >= 0) p.g[m] = static_cast<float>(g);
    acc += g;
    p.gsum[m + r + 1] = static_cast<float>(acc);
  }
}

// Single-word fp16 staging rounds every staged channel value, tap and
// horizontal result to 11 significant bits.  The output is N/D, and D/W is
// the window average of the series phi_hat(f_j - f_i) over the pixel's
// neighbours (Sec. II, first paragraph), so that rounding reaches the
// output divided by D/W.  A series with negative lobes (a crude fit: small
// K for its sigma) drives D/W towards zero wherever the lobes meet the
// image's contrast, and there fp16 misses half an intensity level by far
// (4 levels at K = 2, sigma = 34).  The check: the lowest value of the
// series over one period, relative to its peak.  phi_hat is even and has
// period 2T+1, so t in [0, T + 1/2] covers it; 16 K samples put 32 on
// each period of the highest term, which places the sampled minimum within
// 0.5% of that term's amplitude of the true one.
bool fp16_stage_safe(int K, int T, const double* c) {
  const int n = 16 * K;
  const double half = T + 0.5;
  const double nu = 2.0 * M_PI / (2.0 * T + 1.0);
  double lo = 0.0, hi = 0.0;
  for (int i = 0; i <= n; ++i) {
    const double x = nu * half * i / n;
    // cos(k x) by the three-term recurrence cos((k+1)x) = 2 cos x cos kx - cos((k-1)x)
    const double c1 = std::cos(x);
    double cm = 1.0, ck = c1, v = c[0];
    for (int k = 1; k < K; ++k) {
      v += c[k] * ck;
      const double nx = 2.0 * c1 * ck - cm;
      cm = ck;
      ck = nx;
    }
    if (i == 0) lo = hi = v;
    lo = std::min(lo, v);
    hi = std::max(hi, v);
  }
  return hi > 0.0 && lo >= -kFp16LobeLimit * hi;
}

int effective_prec(int prec, int K, int T, const double* c) {
  if (prec == FOBF_FP16_STAGE && !fp16_stage_safe(K, T, c)) return FOBF_FP16X2_STAGE;
  return prec;
}

fobf_status prec_status(int requested, int used, const char* who) {
  if (requested == used) return FOBF_OK;
  return fail(FOBF_WARN_TOL, std::string(who) +
                                 ": the cosine series dips below -1% of its peak, where "
                                 "single-word fp16 staging loses half an intensity level; "
                                 "ran with two-word fp16 staging (FOBF_FP16X2_STAGE)");
}

fobf_status validate_filter(const float* in, const float* out, int H, int W,
                            int ld_in, int ld_out, double theta, int K, int T,
                            const double* c, int prec, int algo) {
  if (H < 0 || W < 0) return fail(FOBF_EINVAL, "fobf_filter: negative size");
  if (H > 0 && W > 0) {
    if (!in || !out) return fail(FOBF_EINVAL, "fobf_filter: NULL image pointer");
    if (ld_in < W || ld_out < W)
      return fail(FOBF_EINVAL, "fobf_filter: leading dimension below W");
    const char* a0 = reinterpret_cast<const char*>(in);
    const char* a1 = a0 + sizeof(float) * ((static_cast<size_t>(H) - 1) * ld_in + W);
    const char* b0 = reinterpret_cast<const char*>(out);
    const char* b1 = b0 + sizeof(float) * ((static_cast<size_t>(H) - 1) * ld_out + W);
    if (a0 < b1 && b0 < a1)
      return fail(FOBF_EINVAL, "fobf_filter: input and output overlap");
  }
  const int r = spatial_radius(theta);
  if (r < 1) return fail(FOBF_EINVAL, "fobf_filter: theta must be positive and finite");
  if (r > FOBF_RMAX) return fail(FOBF_EINVAL, "fobf_filter: ceil(3 theta) exceeds FOBF_RMAX");
  if (K < 1 || K > FOBF_KMAX) return fail(FOBF_EINVAL, "fobf_filter: K out of range");
  if (T < 1) return fail(FOBF_EINVAL, "fobf_filter: T must be >= 1");
  if (!c) return fail(FOBF_EINVAL, "fobf_filter: c is NULL");
  for (int k = 0; k < K; ++k)
    if (!std::isfinite(c[k])) return fail(FOBF_EINVAL, "fobf_filter: non-finite coefficient");
  if (prec < FOBF_FP32 || prec > FOBF_FP16X2_STAGE)
    return fail(FOBF_EINVAL, "fobf_filter: unknown precision");
  if (algo < FOBF_ALGO_AUTO || algo > FOBF_ALGO_MFMA)
    return fail(FOBF_EINVAL, "fobf_filter: unknown algorithm");
  if (algo == FOBF_ALGO_VALU && prec != FOBF_FP32)
    return fail(FOBF_EINVAL, "fobf_filter: the vector path is float32 only");
  return FOBF_OK;
}

}  // namespace fobf

using namespace fobf;

extern "C" fobf_status fobf_filter(const float* d_in, float* d_out, int H, int W,
                                   int ld_in, int ld_out, double theta, int K,
                                   int T, const double* c, int prec, int algo,
                                   void* hip_stream) {
  fobf_status st = validate_filter(d_in, d_out, H, W, ld_in, ld_out, theta, K,
                                   T, c, prec, algo);
  if (st != FOBF_OK) return st;
  if (H == 0 || W == 0) return FOBF_OK;
  const int eff = effective_prec(prec, K, T, c);
  ImageParams p;
  make_params(p, d_in, d_out, H, W, ld_in, ld_out, theta, K, T, c);
  const int dv = (16 + 2 * p.r + 15) / 16;
  const TuneChoice tc = tuned(eff, dv);
  if (algo == FOBF_ALGO_AUTO) algo = (eff == FOBF_FP32) ? tc.algo : FOBF_ALGO_MFMA;
  if (algo == FOBF_ALGO_VALU) return launch_valu(p, hip_stream);
  st = launch_mfma(p, eff, tc.nblk, hip_stream);
  return st == FOBF_OK ? prec_status(prec, eff, "fobf_filter") : st;
}

extern "C" fobf_status fobf_filter_workspace_size(int H, int W, double theta, int prec,
                                                  size_t* bytes) {
  if (!bytes) return fail(FOBF_EINVAL, "fobf_filter_workspace_size: bytes is NULL");
  if (H < 0 || W < 0) return fail(FOBF_EINVAL, "fobf_filter_workspace_size: negative size");
  const int r = spatial_radius(theta);
  if (r < 1 || r > FOBF_RMAX)
    return fail(FOBF_EINVAL, "fobf_filter_workspace_size: theta out of range");
  if (prec < FOBF_FP32 || prec > FOBF_FP16X2_STAGE)
    return fail(FOBF_EINVAL, "fobf_filter_workspace_size: unknown precision");
  ImageParams p;
  std::memset(&p, 0, sizeof(p));
  p.H = H;
  p.W = W;
  p.r = r;
  // (every precision's workspace form has the same tiles, so a
  // FOBF_FP16_STAGE call that runs as FOBF_FP16X2_STAGE fits it too)
  *bytes = ws_bytes(p, prec);
  return FOBF_OK;
}

extern "C" fobf_status fobf_filter_ws(const float* d_in, float* d_out, int H, int W,
                                      int ld_in, int ld_out, double theta, int K, int T,
                                      const double* c, int prec, int algo, void* d_work,
                                      size_t work_bytes, void* hip_stream) {
  fobf_status st = validate_filter(d_in, d_out, H, W, ld_in, ld_out, theta, K, T, c, prec, algo);
  if (st != FOBF_OK) return st;
  if (H == 0 || W == 0) return FOBF_OK;
  ImageParams p;
  make_params(p, d_in, d_out, H, W, ld_in, ld_out, theta, K, T, c);
  const int eff = effective_prec(prec, K, T, c);
  const size_t need = ws_bytes(p, eff);
  if (need == 0 || algo == FOBF_ALGO_VALU)
    return fobf_filter(d_in, d_out, H, W, ld_in, ld_out, theta, K, T, c, prec, algo,
                       hip_stream);
  if (!d_work || work_bytes < need)
    return fail(FOBF_EINVAL, "fobf_filter_ws: workspace missing or below "
                             "fobf_filter_workspace_size");
  if (reinterpret_cast<uintptr_t>(d_work) % alignof(float) != 0)
    return fail(FOBF_EINVAL, "fobf_filter_ws: workspace not 4-byte aligned");
  const char* w0 = static_cast<const char*>(d_work);
  const char* w1 = w0 + need;
  const char* a0 = reinterpret_cast<const char*>(d_in);
  const char* a1 = a0 + sizeof(float) * ((static_cast<size_t>(H) - 1) * ld_in + W);
  const char* b0 = reinterpret_cast<const char*>(d_out);
  const char* b1 = b0 + sizeof(float) * ((static_cast<size_t>(H) - 1) * ld_out + W);
  if ((w0 < a1 && a0 < w1) || (w0 < b1 && b0 < w1))
    return fail(FOBF_EINVAL, "fobf_filter_ws: workspace overlaps an image");
  st = launch_mfma_ws(p, eff, static_cast<float*>(d_work), hip_stream);
  return st == FOBF_OK ? prec_status(prec, eff, "fobf_filter_ws") : st;
}

extern "C" int fobf_effective_prec(int prec, int K, int T, const double* c) {
  if (prec < FOBF_FP32 || prec > FOBF_FP16X2_STAGE || K < 1 || K > FOBF_KMAX || T < 1 || !c)
    return -1;
  return effective_prec(prec, K, T, c);
}

extern "C" const char* fobf_last_error(void) { return fobf::error_cstr(); }

extern "C" int fobf_version(void) { return 200; }  // 0.2.0
