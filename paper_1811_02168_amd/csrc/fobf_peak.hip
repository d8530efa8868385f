// Instruction-rate probes: the achievable rate of the instruction classes
// the filter kernels are built from, measured on the current device, so
// that roofline fractions can be quoted against a measured ceiling as well
// as against the published one.
#include <hip/hip_runtime.h>

#include <string>

#include "fobf_peak.h"

namespace fobf {
void set_error(const std::string& msg);
}

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;
constexpr int kBlocks = 2048;     // 8 workgroups (32 waves) per CU

// 8 independent fp32 FMA chains per lane (compiled without packed fp32,
// so each is one v_fma_f32 per lane).
__global__ __launch_bounds__(kThreads) void probe_fma(float* out, int iters, float b,
                                                      float c) {
  float a[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = threadIdx.x * 1e-3f + i;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 16; ++u)
#pragma unroll
      for (int i = 0; i < 8; ++i) a[i] = fmaf(a[i], b, c);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += a[i];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// v_sin_f32 throughput: 8 independent chains per lane.
__global__ __launch_bounds__(kThreads) void probe_sin(float* out, int iters) {
  float a[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = threadIdx.x * 1e-4f + 0.01f * i;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 16; ++u)
#pragma unroll
      for (int i = 0; i < 8; ++i) a[i] = __builtin_amdgcn_sinf(a[i]);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += a[i];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// Four independent accumulator chains per wave of one matrix instruction.
template <int KIND>
__global__ __launch_bounds__(kThreads) void probe_mfma(float* out, int iters, float x) {
  f4 acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = f4{0.f, 0.f, 0.f, 0.f};
  const float a = x + threadIdx.x * 1e-6f;
  h8 ah, bh;
  b8 ab, bb;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    ah[j] = static_cast<_Float16>(a);
    bh[j] = static_cast<_Float16>(x);
    ab[j] = static_cast<__bf16>(a);
    bb[j] = static_cast<__bf16>(x);
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if constexpr (KIND == FOBF_PEAK_MFMA_F32)
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, x, acc[i], 0, 0, 0);
        else if constexpr (KIND == FOBF_PEAK_MFMA_F16)
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh, acc[i], 0, 0, 0);
        else
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, bb, acc[i], 0, 0, 0);
      }
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

bool launch(int kind, float* out, int iters, hipStream_t st) {
  const dim3 g(kBlocks), b(kThreads);
  switch (kind) {
    case FOBF_PEAK_VALU_FMA_F32:
      probe_fma<<<g, b, 0, st>>>(out, iters, 0.999f, 1e-3f);
      return true;
    case FOBF_PEAK_VALU_SIN_F32:
      probe_sin<<<g, b, 0, st>>>(out, iters);
      return true;
    case FOBF_PEAK_MFMA_F32:
      probe_mfma<FOBF_PEAK_MFMA_F32><<<g, b, 0, st>>>(out, iters, 1e-3f);
      return true;
    case FOBF_PEAK_MFMA_F16:
      probe_mfma<FOBF_PEAK_MFMA_F16><<<g, b, 0, st>>>(out, iters, 1e-3f);
      return true;
    case FOBF_PEAK_MFMA_BF16:
      probe_mfma<FOBF_PEAK_MFMA_BF16><<<g, b, 0, st>>>(out, iters, 1e-3f);
      return true;
    default:
      return false;
  }
}

// operations counted per loop iteration of one workgroup
double ops_per_iter(int kind) {
  switch (kind) {
    case FOBF_PEAK_VALU_FMA_F32: return 2.0 * 16 * 8 * kThreads;
    case FOBF_PEAK_VALU_SIN_F32: return 1.0 * 16 * 8 * kThreads;
    case FOBF_PEAK_MFMA_F32: return 2.0 * 16 * 16 * 4 * 16 * (kThreads / 64);
    default: return 2.0 * 16 * 16 * 32 * 16 * (kThreads / 64);
  }
}

int iters_for(int kind) {
  switch (kind) {
    case FOBF_PEAK_VALU_FMA_F32: return 2048;
    case FOBF_PEAK_VALU_SIN_F32: return 512;
    case FOBF_PEAK_MFMA_F32: return 1024;
    default: return 2048;
  }
}

}  // namespace

extern "C" fobf_status fobf_peak(int kind, void* stream, double* rate) {
  if (!rate) {
    fobf::set_error("fobf_peak: rate is NULL");
    return FOBF_EINVAL;
  }
  if (kind < FOBF_PEAK_VALU_FMA_F32 || kind > FOBF_PEAK_MFMA_BF16) {
    fobf::set_error("fobf_peak: unknown kind");
    return FOBF_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  fobf_status res = FOBF_EHIP;
  const int iters = iters_for(kind);
  float ms = 0.f;
  if (hipMalloc(&out, sizeof(float) * kBlocks * kThreads) != hipSuccess) {
    fobf::set_error("fobf_peak: hipMalloc failed");
    return FOBF_ENOMEM;
  }
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) goto done;
  launch(kind, out, iters / 8, st);                    // warm-up (clocks, code load)
  if (hipEventRecord(e0, st) != hipSuccess) goto done;
  launch(kind, out, iters, st);
  if (hipGetLastError() != hipSuccess) goto done;
  if (hipEventRecord(e1, st) != hipSuccess) goto done;
  if (hipEventSynchronize(e1) != hipSuccess) goto done;
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess || !(ms > 0.f)) goto done;
  *rate = ops_per_iter(kind) * iters * kBlocks / (ms * 1e-3) / 1e12;
  res = FOBF_OK;
done:
  if (res != FOBF_OK) fobf::set_error("fobf_peak: HIP error while timing the probe");
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipFree(out);
  return res;
}
