// Internal declarations shared by the library's translation units.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/fobf.h"

namespace fobf {

// Number of fobf_prec values (FOBF_FP32 .. FOBF_FP16X2_STAGE): sizes every
// per-precision table and the batch launch counters.
constexpr int kNumPrecisions = FOBF_FP16X2_STAGE + 1;

// Thread-local error message behind fobf_last_error().
void set_error(const std::string& msg);
fobf_status fail(fobf_status st, const std::string& msg);

// Spatial radius ceil(3 theta) computed in double (the oracle does the
// same), or -1 when theta is not positive and finite.
int spatial_radius(double theta);

// Kernel-side parameter block of one image: passed by value to the
// single-image kernels and stored in a device table for batched launches.
struct ImageParams {
  const float* in;
  float* out;
  int H, W, ld_in, ld_out;
  int r;             // spatial radius
  int K;             // order
  float inv_period;  // 1 / (2T + 1)
  int lds_bytes;     // dynamic LDS bytes of the launch (debug-check builds)
  const float* c_dev;       // when set: c_k read from this device array
  float c[FOBF_KMAX];       // c_k in float32
  float g[FOBF_RMAX + 1];   // taps g(0..r); g(-m) = g(m)
  float gsum[2 * FOBF_RMAX + 2];  // gsum[j] = sum_{m=-r}^{j-r-1} g(m), j=0..2r+1
  // debug-check builds (FOBF_CHECKS): the device word collecting violation
  // bits, and the workspace of a workspace-form launch (else null / 0)
  unsigned int* check;
  const float* ws;
  long long ws_floats;
};

// Debug-check builds: the current device's violation word (allocated and
// cleared on first use); null in release builds or when it cannot be made.
unsigned int* check_word();

// Fill an ImageParams from API arguments (validated by the caller).
void make_params(ImageParams& p, const float* in, float* out, int H, int W,
                 int ld_in, int ld_out, double theta, int K, int T,
                 const double* c);

// Single-word fp16 staging is used only for series whose lowest value over
// a period is at least -kFp16LobeLimit times their peak (fobf_api.cpp);
// other FOBF_FP16_STAGE calls run the two-word fp16 kernel instead.
constexpr double kFp16LobeLimit = 0.01;
bool fp16_stage_safe(int K, int T, const double* c);
// The precision a call with `prec` runs in for this series.
int effective_prec(int prec, int K, int T, const double* c);
// FOBF_OK when used == requested, else FOBF_WARN_TOL with the reason set.
fobf_status prec_status(int requested, int used, const char* who);

// Validate fobf_filter arguments; returns FOBF_OK or an error with message.
fobf_status validate_filter(const float* in, const float* out, int H, int W,
                            int ld_in, int ld_out, double theta, int K, int T,
                            const double* c, int prec, int algo);

// Launchers (fobf_valu.hip / fobf_mfma.hip).  nblk = 16-row blocks per
// tile (tile height 16 nblk).  Return FOBF_EHIP on launch failure with the
// message set.
fobf_status launch_valu(const ImageParams& p, void* stream);
fobf_status launch_mfma(const ImageParams& p, int prec, int nblk, void* stream);
// Workspace form (fobf_filter_ws): tile height in 16-row blocks (0: not
// used for this image and precision), workspace bytes it needs, launch.
int ws_nblk(const ImageParams& p, int prec);
size_t ws_bytes(const ImageParams& p, int prec);
fobf_status launch_mfma_ws(const ImageParams& p, int prec, float* work, void* stream);

// Tuning table (fobf_tune.cpp): per precision and radius class dv =
// ceil((16 + 2r) / 16), the algorithm and tile height chosen by
// fobf_autotune, or the built-in defaults.
struct TuneChoice {
  int algo;   // FOBF_ALGO_VALU or FOBF_ALGO_MFMA
  int nblk;   // 16-row blocks per tile
};
TuneChoice tuned(int prec, int dv);
int batch_tile_blocks(int prec, int dv, int H);

// Copies host bytes to the device on `stream` through a library-owned
// pinned staging buffer, so the caller's host memory may be reused as soon
// as this returns.  Never synchronises.
fobf_status upload_async(void* dst, const void* src, size_t bytes, void* stream);

}  // namespace fobf
