// Tile-shape autotuner, its table, and the pinned upload staging pool.
//
// The table holds, per precision and radius class dv = ceil((16+2r)/16),
// the algorithm (float32 only: matrix cores or vector ALU) and the tile
// height (16-row blocks) that fobf_filter uses, and that the batch kernel
// uses (capped at 8 blocks and at the image height).  fobf_autotune fills
// it by timing every candidate on the device; fobf_tune_save / _load keep
// it across processes as a small text file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fobf_internal.h"

namespace fobf {
namespace {

constexpr int kPrecs = kNumPrecisions;
constexpr int kDvMax = 7;   // dv for r = FOBF_RMAX = 48

struct Slot {
  TuneChoice c;
  float ms;      // measured time of the choice (0 when built in)
  bool set;
};

std::mutex g_tune_mu;
Slot g_table[kPrecs][kDvMax + 1];

// Defaults measured on MI355X at 4096^2, r = 30: fp32 8 blocks (1.83 ms vs
// 1.95 at 6, 2.15 at 4; taller tiles drop to one workgroup per CU), fp16
// and bf16 8 blocks (fp16 0.78 ms, bf16 1.62 ms vs 1.78 at 6).  Staged
// launches cap the height at what fits in LDS.
TuneChoice builtin(int prec, int dv) {
  (void)prec;
  (void)dv;
  return {FOBF_ALGO_MFMA, 8};
}

// deterministic 0..255 test pattern for the tuning image
__global__ void fill_pattern(float* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = static_cast<float>((i * 2654435761u >> 13) & 255u);
}

}  // namespace

TuneChoice tuned(int prec, int dv) {
  if (prec < 0 || prec >= kPrecs || dv < 0 || dv > kDvMax) return builtin(prec, dv);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const Slot& s = g_table[prec][dv];
  return s.set ? s.c : builtin(prec, dv);
}

int batch_tile_blocks(int prec, int dv, int H) {
  const int nb = tuned(prec, dv).nblk;
  return std::max(1, std::min({nb, 8, (H + 15) / 16}));
}

// ------------------------------------------------------- upload staging --

namespace {
struct Staging {
  void* host;
  size_t cap;
  hipEvent_t done;
  int device;
  bool busy;
};
std::mutex g_stage_mu;
std::vector<Staging> g_stage;
}  // namespace

fobf_status upload_async(void* dst, const void* src, size_t bytes, void* stream) {
  if (bytes == 0) return FOBF_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FOBF_EHIP, "upload: hipGetDevice failed");
  std::lock_guard<std::mutex> lk(g_stage_mu);
  Staging* use = nullptr;
  for (Staging& s : g_stage) {
    if (s.device != dev || s.cap < bytes) continue;
    if (s.busy && hipEventQuery(s.done) != hipSuccess) continue;
    use = &s;
    break;
  }
  if (!use) {
    Staging s{};
    s.cap = std::max<size_t>(bytes, 64 << 10);
    s.device = dev;
    if (hipHostMalloc(&s.host, s.cap, hipHostMallocDefault) != hipSuccess)
      return fail(FOBF_ENOMEM, "upload: pinned staging allocation failed");
    if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) {
      hipHostFree(s.host);
      return fail(FOBF_EHIP, "upload: event creation failed");
    }
    g_stage.push_back(s);
    use = &g_stage.back();
  }
  std::memcpy(use->host, src, bytes);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(dst, use->host, bytes, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipEventRecord(use->done, st);
  use->busy = true;
  if (e != hipSuccess) return fail(FOBF_EHIP, std::string("upload: ") + hipGetErrorString(e));
  return FOBF_OK;
}

}  // namespace fobf

using namespace fobf;

extern "C" fobf_status fobf_autotune(int prec, int H, int W, int K, void* hip_stream) {
  if (prec < FOBF_FP32 || prec > FOBF_FP16X2_STAGE)
    return fail(FOBF_EINVAL, "fobf_autotune: unknown precision");
  if (H < 16 || W < 16 || K < 1 || K > FOBF_KMAX)
    return fail(FOBF_EINVAL, "fobf_autotune: need H, W >= 16 and 1 <= K <= FOBF_KMAX");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  float *in = nullptr, *out = nullptr;
  const size_t n = static_cast<size_t>(H) * W;
  if (hipMalloc(&in, n * sizeof(float)) != hipSuccess ||
      hipMalloc(&out, n * sizeof(float)) != hipSuccess) {
    if (in) hipFree(in);
    return fail(FOBF_ENOMEM, "fobf_autotune: device allocation failed");
  }
  hipLaunchKernelGGL(fill_pattern, dim3((n + 255) / 256), dim3(256), 0, st, in, static_cast<int>(n));
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  std::vector<double> c(K, 0.0);
  c[0] = 0.4;
  for (int k = 1; k < K; ++k) c[k] = 0.6 / (K - 1);
  fobf_status result = FOBF_OK;
  for (int dv = 2; dv <= kDvMax && result == FOBF_OK; ++dv) {
    const int r = std::min(FOBF_RMAX, 8 * (dv - 1));
    const double theta = r / 3.0;
    ImageParams p;
    make_params(p, in, out, H, W, W, W, theta, K, 150, c.data());
    struct Cand {
      int algo, nblk;
    };
    std::vector<Cand> cands;
    for (int nb : {2, 4, 8, 16}) cands.push_back({FOBF_ALGO_MFMA, nb});
    if (prec == FOBF_FP32) cands.push_back({FOBF_ALGO_VALU, 0});
    float best = 1e30f;
    TuneChoice bestc = builtin(prec, dv);
    for (const Cand& cd : cands) {
      auto launch = [&]() {
        return cd.algo == FOBF_ALGO_VALU ? launch_valu(p, st) : launch_mfma(p, prec, cd.nblk, st);
      };
      if (launch() != FOBF_OK) continue;   // e.g. a shape that does not fit LDS
      hipEventRecord(e0, st);
      const int reps = 3;
      for (int i = 0; i < reps; ++i) launch();
      hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) {
        result = fail(FOBF_EHIP, "fobf_autotune: timing failed");
        break;
      }
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      ms /= reps;
      if (ms < best) {
        best = ms;
        bestc = {cd.algo, cd.algo == FOBF_ALGO_VALU ? 8 : cd.nblk};
      }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_table[prec][dv] = {bestc, best, true};
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipStreamSynchronize(st);
  hipFree(in);
  hipFree(out);
  return result;
}

extern "C" fobf_status fobf_tune_save(const char* path) {
  if (!path) return fail(FOBF_EINVAL, "fobf_tune_save: path is NULL");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(FOBF_EINVAL, std::string("fobf_tune_save: cannot open ") + path);
  std::fprintf(f, "# fobf tuning table v1: prec dv algo nblk ms\n");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (int pr = 0; pr < kPrecs; ++pr)
    for (int dv = 0; dv <= kDvMax; ++dv) {
      const Slot& s = g_table[pr][dv];
      if (s.set) std::fprintf(f, "%d %d %d %d %.6f\n", pr, dv, s.c.algo, s.c.nblk, s.ms);
    }
  std::fclose(f);
  return FOBF_OK;
}

extern "C" fobf_status fobf_tune_load(const char* path) {
  if (!path) return fail(FOBF_EINVAL, "fobf_tune_load: path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(FOBF_EINVAL, std::string("fobf_tune_load: cannot open ") + path);
  char line[256];
  int loaded = 0;
  std::vector<std::pair<std::pair<int, int>, Slot>> rows;
  while (std::fgets(line, sizeof(line), f)) {
    if (line[0] == '#') continue;
    int pr, dv, algo, nb;
    float ms;
    if (std::sscanf(line, "%d %d %d %d %f", &pr, &dv, &algo, &nb, &ms) != 5) continue;
    if (pr < 0 || pr >= kPrecs || dv < 0 || dv > kDvMax) continue;
    if (algo != FOBF_ALGO_MFMA && !(algo == FOBF_ALGO_VALU && pr == FOBF_FP32)) continue;
    if (nb < 1 || nb > 16) continue;
    rows.push_back({{pr, dv}, Slot{{algo, nb}, ms, true}});
  }
  std::fclose(f);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& r : rows) {
    g_table[r.first.first][r.first.second] = r.second;
    ++loaded;
  }
  if (loaded == 0) return fail(FOBF_EINVAL, "fobf_tune_load: no valid rows");
  return FOBF_OK;
}

extern "C" fobf_status fobf_tune_reset(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& row : g_table)
    for (auto& s : row) s.set = false;
  return FOBF_OK;
}

extern "C" fobf_status fobf_tune_get(int prec, double theta, int* algo, int* nblk) {
  const int r = spatial_radius(theta);
  if (r < 1 || r > FOBF_RMAX || prec < 0 || prec >= kPrecs || !algo || !nblk)
    return fail(FOBF_EINVAL, "fobf_tune_get: bad argument");
  const TuneChoice c = tuned(prec, (16 + 2 * r + 15) / 16);
  *algo = c.algo;
  *nblk = c.nblk;
  return FOBF_OK;
}
