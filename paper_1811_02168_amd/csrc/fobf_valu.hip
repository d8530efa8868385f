// Vector-ALU path of the K-term shiftable bilateral filter (float32).
//
// The filter (Sec. II, first paragraph, with eq. (3) as range kernel) is a
// sum over channels X of spatial convolutions, each weighted per output
// pixel:
//   channel          weight at output pixel i     accumulates into
//   f                c_0                          N
//   1 (in-image)     c_0                          D
//   C_k f, S_k f     c_k C_k(i), c_k S_k(i)       N      (k = 1..K-1)
//   C_k,   S_k       c_k C_k(i), c_k S_k(i)       D
// with C_k = cos(2 pi k f / (2T+1)), S_k = sin(...); out = N / D.
//
// One workgroup owns a TX x TY output tile.  For each channel it builds the
// channel over the tile plus an r-halo in LDS (out-of-image pixels are 0 in
// every channel: excluded neighbours), runs the horizontal pass into LDS,
// then the vertical pass in registers, and folds the result into the
// per-pixel N and D accumulators, which never leave registers.  Nothing but
// f (read) and the output (written once) touches HBM.
#include <hip/hip_runtime.h>

#include "fobf_internal.h"

#ifndef FOBF_CHECKS
#define FOBF_CHECKS 0
#endif

namespace fobf {
namespace {

constexpr int VTX = 32;        // output tile width
constexpr int VTY = 32;        // output tile height
constexpr int VTHREADS = 256;  // 4 waves

// Row pitch of the channel tile: >= IW and = 1 (mod 32), so that the 8
// lanes of a row (stride 4 floats) and 4 consecutive rows hit distinct
// banks.
__host__ __device__ inline int valu_pitch(int r) {
  int iw = VTX + 2 * r + 4;  // +4: the sliding window reads 4 past the end
  return ((iw + 30) / 32) * 32 + 1;
}

__host__ inline size_t valu_lds_bytes(int r) {
  const int ih = VTY + 2 * r;
  return sizeof(float) * (static_cast<size_t>(ih) * valu_pitch(r)   // channel
                          + static_cast<size_t>(ih + 4) * VTX       // H pass
                          + (2 * r + 1) + 4);                        // taps
}

// cos and sin of 2 pi * x for x in revolutions, reduced to [0, 1) first.
__device__ inline void sincos_rev(float x, float* s, float* c) {
  const float t = x - floorf(x);
  *s = __builtin_amdgcn_sinf(t);
  *c = __builtin_amdgcn_cosf(t);
}

__global__ __launch_bounds__(VTHREADS) void valu_kernel(ImageParams p) {
  extern __shared__ float lds[];
  const int r = p.r;
  const int IH = VTY + 2 * r;
  const int P = valu_pitch(r);
  float* xS = lds;                    // IH x P channel tile
  float* hS = xS + IH * P;            // (IH + 4) x VTX horizontal pass
  float* gS = hS + (IH + 4) * VTX;    // 2r+1 taps g(-r..r)

  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * VTX;
  const int y0 = blockIdx.y * VTY;
#if FOBF_CHECKS
  // debug-check build: LDS starts as NaN words; the sliding windows' last
  // reads (row xb + 2r + 4 of the channel tile, row oy0 + 2r + 4 of the
  // horizontal pass) stay inside the allocation
  for (int i = tid; i < p.lds_bytes / 4; i += VTHREADS) reinterpret_cast<uint32_t*>(lds)[i] = ~0u;
  __syncthreads();
  if (p.check) {
    const long long need = sizeof(float) * (static_cast<long long>(IH) * P + (IH + 4) * VTX +
                                            2 * r + 1);
    if (need > p.lds_bytes || VTX - 4 + 2 * r + 4 >= P ||
        (VTY - 4) + 2 * r + 4 >= IH + 4)
      atomicOr(p.check, FOBF_CHECK_LDS);
  }
#endif
  for (int m = tid; m <= 2 * r; m += VTHREADS) gS[m] = p.g[m <= r ? r - m : m - r];

  // output pixels of this thread: column ox, rows oy0 .. oy0+3
  const int ox = tid % VTX;
  const int oy0 = (tid / VTX) * 4;
  float fo[4], N[4], D[4];
  {
    const int gx = x0 + ox;
    // W(i) = Wy(y) Wx(x): sum of the in-image taps (blur of the ones)
    float wx = 0.f;
    if (gx < p.W) {
      const int lo = max(-r, gx - p.W + 1), hi = min(r, gx);
      wx = p.gsum[hi + r + 1] - p.gsum[lo + r];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int gy = y0 + oy0 + i;
      const bool in = gx < p.W && gy < p.H;
      fo[i] = in ? p.in[static_cast<size_t>(gy) * p.ld_in + gx] : 0.f;
      float wy = 0.f;
      if (gy < p.H) {
        const int lo = max(-r, gy - p.H + 1), hi = min(r, gy);
        wy = p.gsum[hi + r + 1] - p.gsum[lo + r];
      }
      N[i] = 0.f;
      D[i] = p.c[0] * wx * wy;
    }
  }

  const int nch = 1 + 4 * (p.K - 1);
  for (int ch = 0; ch < nch; ++ch) {
    // channel id: 0 -> f; otherwise k = (ch-1)/4 + 1, j = (ch-1)%4:
    // j=0 C f, j=1 S f, j=2 C, j=3 S
    const int k = ch == 0 ? 0 : (ch - 1) / 4 + 1;
    const int j = ch == 0 ? 0 : (ch - 1) % 4;

    // 1. channel over tile + halo
    for (int idx = tid; idx < IH * P; idx += VTHREADS) {
      const int yy = idx / P, xx = idx - yy * P;
      const int gy = y0 - r + yy, gx = x0 - r + xx;
      float v = 0.f;
      if (xx < VTX + 2 * r && gy >= 0 && gy < p.H && gx >= 0 && gx < p.W) {
        const float f = p.in[static_cast<size_t>(gy) * p.ld_in + gx];
        if (k == 0) {
          v = f;
        } else {
          float s, c;
          sincos_rev(static_cast<float>(k) * f * p.inv_period, &s, &c);
          v = (j == 0) ? c * f : (j == 1) ? s * f : (j == 2) ? c : s;
        }
      }
      xS[idx] = v;
    }
    __syncthreads();

    // 2. horizontal pass: hS(y, x) = sum_m g(m) X(y, x + m), 4 outputs/item
    for (int item = tid; item < IH * (VTX / 4); item += VTHREADS) {
      const int yy = item / (VTX / 4);
      const int xb = (item % (VTX / 4)) * 4;
      const float* row = xS + yy * P + xb;
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
      float w0 = row[0], w1 = row[1], w2 = row[2], w3 = row[3];
      for (int m = 0; m <= 2 * r; ++m) {
        const float gm = gS[m];
        a0 = fmaf(gm, w0, a0);
        a1 = fmaf(gm, w1, a1);
        a2 = fmaf(gm, w2, a2);
        a3 = fmaf(gm, w3, a3);
        w0 = w1;
        w1 = w2;
        w2 = w3;
        w3 = row[m + 4];
      }
      float* h = hS + yy * VTX + xb;
      h[0] = a0;
      h[1] = a1;
      h[2] = a2;
      h[3] = a3;
    }
    __syncthreads();

    // 3. vertical pass for this thread's 4 pixels, then fold into N / D
    {
      const float* col = hS + oy0 * VTX + ox;
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
      float w0 = col[0], w1 = col[VTX], w2 = col[2 * VTX], w3 = col[3 * VTX];
      for (int m = 0; m <= 2 * r; ++m) {
        const float gm = gS[m];
        a0 = fmaf(gm, w0, a0);
        a1 = fmaf(gm, w1, a1);
        a2 = fmaf(gm, w2, a2);
        a3 = fmaf(gm, w3, a3);
        w0 = w1;
        w1 = w2;
        w2 = w3;
        w3 = col[(m + 4) * VTX];
      }
      const float a[4] = {a0, a1, a2, a3};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (k == 0) {
          N[i] = fmaf(p.c[0], a[i], N[i]);
        } else {
          float s, c;
          sincos_rev(static_cast<float>(k) * fo[i] * p.inv_period, &s, &c);
          const float w = p.c[k] * ((j == 0 || j == 2) ? c : s);
          if (j < 2)
            N[i] = fmaf(w, a[i], N[i]);
          else
            D[i] = fmaf(w, a[i], D[i]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gy = y0 + oy0 + i, gx = x0 + ox;
    if (gy < p.H && gx < p.W) {
#if FOBF_CHECKS
      if (p.check && gx >= p.ld_out) atomicOr(p.check, FOBF_CHECK_OUT);
#endif
      p.out[static_cast<size_t>(gy) * p.ld_out + gx] = N[i] / D[i];
    }
  }
}

}  // namespace

fobf_status launch_valu(const ImageParams& p, void* stream) {
  const size_t lds = valu_lds_bytes(p.r);
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&valu_kernel),
      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)attr;
  dim3 grid((p.W + VTX - 1) / VTX, (p.H + VTY - 1) / VTY);
  ImageParams q = p;
  q.lds_bytes = static_cast<int>(lds);
  hipLaunchKernelGGL(valu_kernel, grid, dim3(VTHREADS), lds,
                     static_cast<hipStream_t>(stream), q);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(FOBF_EHIP, std::string("valu_kernel launch: ") + hipGetErrorString(e));
  return FOBF_OK;
}

}  // namespace fobf
