// Matrix-core (MFMA) path of the K-term shiftable bilateral filter.
//
// Each spatial convolution of a channel X with the separable truncated
// Gaussian is written as two banded Toeplitz products and run on the
// 16x16x4 float32 matrix instruction:
//
//   horizontal  Hx[y][x] = sum_c X[y][c] Gh[c][x],  Gh[c][x] = g(c - x)
//   vertical    V[y][x]  = sum_h Gv[y][h] Hx[h][x], Gv[y][h] = g(h - y)
//
// A wave owns a strip of 16 output columns and walks down it in blocks of
// 16 rows.  For every 16-row block of the horizontal pass it streams the
// 16 + 2r input columns in steps of 4 (A operand = channel values, built on
// the fly from f: trig is never stored), multiplying by a constant slice of
// Gh held in registers.  The 16x16 result is left in the accumulator layout
// (lane l, register v holds row 4*(l/16)+v, column l%16), which is exactly
// a B operand of the vertical product if the contraction index k of that
// product enumerates rows {v, 4+v, 8+v, 12+v}; the vertical Toeplitz slices
// are pre-permuted to match, so the horizontal result feeds the vertical
// pass straight from registers.  A ring of DV horizontal blocks (DV =
// ceil((16 + 2r) / 16)) holds what one 16-row vertical output block needs.
//
// Channels are processed in groups that share one trig evaluation (the four
// channels C f, S f, C, S of one frequency k, plus f itself with k = 1).
// After the vertical pass the group's contribution is weighted with the
// trig values of the output pixel and added into per-pixel N and D sums
// kept in LDS; the output N / D is written once at the end.
#include <hip/hip_runtime.h>

#include "fobf_internal.h"

namespace fobf {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int MWAVES = 4;               // waves per workgroup (x strips)
constexpr int MTHREADS = 64 * MWAVES;
constexpr int MSTRIP = 16;              // output columns per wave

__device__ inline void sincos_rev(float x, float* s, float* c) {
  const float t = x - floorf(x);
  *s = __builtin_amdgcn_sinf(t);
  *c = __builtin_amdgcn_cosf(t);
}

__device__ inline float tap(const float* gS, int d, int r) {
  return (d >= -r && d <= r) ? gS[d < 0 ? -d : d] : 0.f;
}

// One channel group over the whole strip.  G = 1: {f};  G = 4: {C f, S f,
// C, S} of frequency k;  G = 5: {f, C f, S f, C, S} with frequency k.
template <int DV, int G>
__device__ void strip_group(const ImageParams& p, int k, int x0w, int y0,
                            int nblk, const float* gS, float* Ns, float* Ds,
                            int lane) {
  const int r = p.r;
  const int SH = (MSTRIP + 2 * r + 3) / 4;   // horizontal K-steps (<= 4*DV)
  const int li = lane & 15;                  // A row / B,D column
  const int lk = lane >> 4;                  // A,B contraction index
  const float kinv = static_cast<float>(k) * p.inv_period;

  // constant operands: horizontal slices Bh[s] and vertical slices Av[d][v]
  float Bh[4 * DV];
#pragma unroll
  for (int s = 0; s < 4 * DV; ++s) Bh[s] = tap(gS, 4 * s + lk - r - li, r);
  float Av[DV][4];
#pragma unroll
  for (int d = 0; d < DV; ++d)
#pragma unroll
    for (int v = 0; v < 4; ++v) Av[d][v] = tap(gS, 16 * d + 4 * lk + v - r - li, r);

  f4 ring[DV][G];
  const int QB = nblk + DV - 1;   // horizontal blocks covering the strip
  const int colbase = x0w - r + lk;

  for (int qq = 0; qq < QB; qq += DV) {
#pragma unroll
    for (int u = 0; u < DV; ++u) {
      const int q = qq + u;
      if (q < QB) {
        // ---- horizontal pass for H rows 16q .. 16q+15 ----
        const int row = y0 - r + 16 * q + li;
        const bool rowok = row >= 0 && row < p.H;
        const float* rp = p.in + static_cast<size_t>(rowok ? row : 0) * p.ld_in;
        f4 acc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 4 * DV; ++s) {
          if (s < SH) {
            const int col = colbase + 4 * s;
            const bool ok = rowok && col >= 0 && col < p.W;
            const float fv = ok ? rp[col] : 0.f;
            float a[G];
            if (G == 1) {
              a[0] = fv;
            } else {
              float sn, cs;
              sincos_rev(kinv * fv, &sn, &cs);
              const float m = ok ? 1.f : 0.f;
              const int o = (G == 5) ? 1 : 0;
              if (G == 5) a[0] = fv;
              a[o + 0] = cs * fv;
              a[o + 1] = sn * fv;
              a[o + 2] = cs * m;
              a[o + 3] = sn * m;
            }
#pragma unroll
            for (int g = 0; g < G; ++g)
              acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[g], Bh[s], acc[g], 0, 0, 0);
          }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) ring[u][g] = acc[g];

        // ---- vertical pass for output block pb = q - DV + 1 ----
        const int pb = q - (DV - 1);
        if (pb >= 0) {
          f4 vacc[G];
#pragma unroll
          for (int g = 0; g < G; ++g) vacc[g] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int d = 0; d < DV; ++d) {
            const int slot = (u + 1 + d) % DV;
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
              for (int g = 0; g < G; ++g)
                vacc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(Av[d][v], ring[slot][g][v],
                                                               vacc[g], 0, 0, 0);
          }
          // ---- fold into N, D at the output pixels ----
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int orow = 16 * pb + 4 * lk + v;       // row within strip
            const int gy = y0 + orow, gx = x0w + li;
            const bool in = gy < p.H && gx < p.W;
            const float fo = in ? p.in[static_cast<size_t>(gy) * p.ld_in + gx] : 0.f;
            const int idx = orow * MSTRIP + li;
            float n = Ns[idx], dd = Ds[idx];
            if (G == 1) {
              n = fmaf(p.c[0], vacc[0][v], n);
            } else {
              float sn, cs;
              sincos_rev(kinv * fo, &sn, &cs);
              const int o = (G == 5) ? 1 : 0;
              const float ck = p.c[k];
              if (G == 5) n = fmaf(p.c[0], vacc[0][v], n);
              n = fmaf(ck, fmaf(cs, vacc[o + 0][v], sn * vacc[o + 1][v]), n);
              dd = fmaf(ck, fmaf(cs, vacc[o + 2][v], sn * vacc[o + 3][v]), dd);
            }
            Ns[idx] = n;
            Ds[idx] = dd;
          }
        }
      }
    }
  }
}

template <int DV>
__global__ __launch_bounds__(MTHREADS) void mfma_f32_kernel(ImageParams p, int nblk) {
  extern __shared__ float lds[];
  const int r = p.r;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int TYo = 16 * nblk;
  float* gS = lds;                                    // taps g(0..r)
  float* Ns = lds + 64 + wave * 2 * TYo * MSTRIP;     // this wave's N
  float* Ds = Ns + TYo * MSTRIP;                      // this wave's D
  for (int m = threadIdx.x; m <= r; m += MTHREADS) gS[m] = p.g[m];

  const int x0w = blockIdx.x * (MWAVES * MSTRIP) + wave * MSTRIP;
  const int y0 = blockIdx.y * TYo;

  // N = 0, D = c_0 W(i) with W(i) = Wy(y) Wx(x) the in-image tap sums
  {
    const int gx = x0w + (lane & 15);
    float wx = 0.f;
    if (gx < p.W) {
      const int lo = max(-r, gx - p.W + 1), hi = min(r, gx);
      wx = p.gsum[hi + r + 1] - p.gsum[lo + r];
    }
    for (int row = lane >> 4; row < TYo; row += 4) {
      const int gy = y0 + row;
      float wy = 0.f;
      if (gy < p.H) {
        const int lo = max(-r, gy - p.H + 1), hi = min(r, gy);
        wy = p.gsum[hi + r + 1] - p.gsum[lo + r];
      }
      Ns[row * MSTRIP + (lane & 15)] = 0.f;
      Ds[row * MSTRIP + (lane & 15)] = p.c[0] * wx * wy;
    }
  }
  __syncthreads();

  if (p.K == 1) {
    strip_group<DV, 1>(p, 0, x0w, y0, nblk, gS, Ns, Ds, lane);
  } else {
    strip_group<DV, 5>(p, 1, x0w, y0, nblk, gS, Ns, Ds, lane);
    for (int k = 2; k < p.K; ++k) strip_group<DV, 4>(p, k, x0w, y0, nblk, gS, Ns, Ds, lane);
  }

  for (int row = lane >> 4; row < TYo; row += 4) {
    const int gy = y0 + row, gx = x0w + (lane & 15);
    if (gy < p.H && gx < p.W) {
      const int idx = row * MSTRIP + (lane & 15);
      p.out[static_cast<size_t>(gy) * p.ld_out + gx] = Ns[idx] / Ds[idx];
    }
  }
}

template <int DV>
fobf_status launch_dv(const ImageParams& p, int nblk, void* stream) {
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&mfma_f32_kernel<DV>),
      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  (void)attr;
  const size_t lds = sizeof(float) * (64 + static_cast<size_t>(MWAVES) * 2 * 16 * nblk * MSTRIP);
  dim3 grid((p.W + MWAVES * MSTRIP - 1) / (MWAVES * MSTRIP), (p.H + 16 * nblk - 1) / (16 * nblk));
  hipLaunchKernelGGL(mfma_f32_kernel<DV>, grid, dim3(MTHREADS), lds,
                     static_cast<hipStream_t>(stream), p, nblk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(FOBF_EHIP, std::string("mfma_f32_kernel launch: ") + hipGetErrorString(e));
  return FOBF_OK;
}

}  // namespace

fobf_status launch_mfma(const ImageParams& p, int prec, void* stream) {
  if (prec != FOBF_FP32)
    return fail(FOBF_EINVAL, "fobf_filter: staged precisions not built yet");
  const int DV = (MSTRIP + 2 * p.r + 15) / 16;
  const int nblk = 8;
  switch (DV) {
    case 2: return launch_dv<2>(p, nblk, stream);
    case 3: return launch_dv<3>(p, nblk, stream);
    case 4: return launch_dv<4>(p, nblk, stream);
    case 5: return launch_dv<5>(p, nblk, stream);
    case 6: return launch_dv<6>(p, nblk, stream);
    case 7: return launch_dv<7>(p, nblk, stream);
    default: return fail(FOBF_EINVAL, "fobf_filter: radius out of range for MFMA path");
  }
}

int auto_algo(int r, int K, int prec) {
  (void)r;
  (void)K;
  (void)prec;
  return FOBF_ALGO_MFMA;
}

}  // namespace fobf
