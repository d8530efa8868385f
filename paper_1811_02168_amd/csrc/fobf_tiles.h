#pragma once
// Device building blocks of the matrix-core filter, shared by the
// single-image kernels (fobf_mfma.hip) and the persistent batch kernel
// (fobf_batch.hip).
//
// Matrix-core (MFMA) paths of the K-term shiftable bilateral filter.
//
// The filter (Sec. II, first paragraph, with the cosine series of eq. (3)
// as range kernel) is a sum over channels X of truncated-Gaussian spatial
// convolutions, each weighted per output pixel i:
//   channel        weight at i        into     (C_k = cos(2 pi k f/(2T+1)),
//   f              c_0                N         S_k = sin(...), k = 1..K-1)
//   C_k f, S_k f   c_k C_k(i), S_k(i) N
//   C_k,   S_k     c_k C_k(i), S_k(i) D,   plus D += c_0 W(i), out = N / D.
// Neighbours outside the image are excluded (every channel zero padded);
// W(i) = Wy(y) Wx(x) is the sum of the in-image taps.
//
// Each convolution is two banded Toeplitz products on the matrix cores:
//   horizontal  H[y][x] = sum_c X[y][c] Gh[c][x],  Gh[c][x] = g(c - x)
//   vertical    V[y][x] = sum_h Gv[y][h] H[h][x],  Gv[y][h] = g(h - y)
// A wave owns a strip of 16 output columns and walks down it in blocks of
// 16 rows.  The 16x16 horizontal result sits in the accumulator layout
// (lane l, element v = row 4*(l/16)+v, column l%16).  That is already a B
// operand of the vertical product once its contraction index is taken to
// enumerate those rows; the vertical Toeplitz slices are built for that
// order, so H never leaves registers.  A ring of DV = ceil((16+2r)/16)
// horizontal blocks holds what one vertical output block needs.
//
// float32 path (16x16x4 f32): channel values are built on the fly from f
//   in each lane (trig never stored); N, D live in LDS.
// staged paths (16x16x32 f16 / bf16, f32 accumulation): the workgroup
//   builds each 16-row block of channels once into LDS in the staging
//   type (shared by all its strips) -- one fp16 word, or hi + lo words of
//   bf16 or fp16 -- horizontal results are rounded the same way for the
//   vertical product; N and D live in LDS.
// workspace forms (every precision): N and D of each tile live in a device
//   workspace instead, which frees the LDS for 512-row tiles; float32 then
//   stages its channels once per workgroup too (float32 words, the same
//   sums in the same order as the per-lane path).
// In all of them channel f (k = 0) forms a group of its own without trig
// (merged with frequency 1 in the float32 and fp16 workspace forms), and
// every k >= 1 forms a group of four channels sharing one sin/cos.



#include <hip/hip_runtime.h>

#include <atomic>

#include "fobf_internal.h"

#ifndef FOBF_CHECKS
#define FOBF_CHECKS 0
#endif

namespace fobf {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef __bf16 bh4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

constexpr int MWAVES = 4;             // waves per workgroup = x strips
constexpr int MTHREADS = 64 * MWAVES;
constexpr int MSTRIP = 16;            // output columns per wave
// LDS table (floats): taps g(0..r) at 0, c_k at 64, tap prefix sums at 96;
// 256 floats keep what follows 16-byte aligned.
constexpr int LDS_TABLE = 256;

__device__ __forceinline__ void sincos_rev(float x, float* s, float* c) {
  const float t = __builtin_amdgcn_fractf(x);
  *s = __builtin_amdgcn_sinf(t);
  *c = __builtin_amdgcn_cosf(t);
}

// An LDS pointer held in one register as it stands: the compiler may not
// split it into a variable part plus a constant (which, when the constant
// exceeds the 1 KB reach of the ds_read2 offset fields, costs one vector
// add per read); the reads through it then take their small constant
// offsets in the instruction's offset fields.
template <typename T>
__device__ __forceinline__ T* lds_pinned(T* p) {
  auto q = (__attribute__((address_space(3))) T*)p;
  asm("" : "+v"(q));
  return (T*)q;
}

__device__ __forceinline__ float tap(const float* gS, int d, int r) {
  return (d >= -r && d <= r) ? gS[d < 0 ? -d : d] : 0.f;
}

// in-image tap sum along one axis at coordinate x of an axis of length n
__device__ __forceinline__ float edge_weight(const float* gsumS, int x, int n, int r) {
  if (x < 0 || x >= n) return 0.f;
  const int lo = max(-r, x - n + 1), hi = min(r, x);
  return gsumS[hi + r + 1] - gsumS[lo + r];
}

// Scalars of one image, plus the LDS tables (taps g(0..r), c_k, prefix
// sums of the taps) shared by the workgroup.
struct Img {
  const float* __restrict__ in;
  float* __restrict__ out;
  int H, W, ld_in, ld_out, r, K;
  float inv_period;
#if FOBF_CHECKS
  unsigned int* check;
  const float* ws;
  long long ws_floats;
  int lds_bytes;
#endif
};

// The Img of a parameter block.  A macro for the reason FOBF_LOAD_TABLES is
// one (the block is indexed where it is, never passed by address).
#if FOBF_CHECKS
#define FOBF_IMG(p)                                                                   \
  Img{(p).in, (p).out, (p).H, (p).W, (p).ld_in, (p).ld_out, (p).r, (p).K,             \
      (p).inv_period, (p).check, (p).ws, (p).ws_floats, (p).lds_bytes}
#else
#define FOBF_IMG(p)                                                                   \
  Img{(p).in, (p).out, (p).H, (p).W, (p).ld_in, (p).ld_out, (p).r, (p).K, (p).inv_period}
#endif

// ---- debug-check builds (FOBF_CHECKS = 1) --------------------------------
// Every check reads only: a failed one ORs its FOBF_CHECK_* bit into the
// image's violation word (a vector atomic) and the kernel carries on, so
// the checked kernels compute what the release kernels compute.  In
// release builds all of this compiles to nothing.
#if FOBF_CHECKS
#define FOBF_CHK(im, cond, bit)                                     \
  do {                                                              \
    if (!(cond) && (im).check) atomicOr((im).check, (bit));         \
  } while (0)
#else
#define FOBF_CHK(im, cond, bit) \
  do {                          \
  } while (0)
#endif

// `bytes` at p lie inside the launch's dynamic LDS allocation.
__device__ __forceinline__ void chk_lds(const Img& im, const void* p, int bytes) {
#if FOBF_CHECKS
  extern __shared__ float fobf_dyn_lds[];
  const long long off =
      static_cast<const char*>(p) - reinterpret_cast<const char*>(fobf_dyn_lds);
  FOBF_CHK(im, off >= 0 && off + bytes <= im.lds_bytes, FOBF_CHECK_LDS);
#endif
}

// (row, col) is a pixel of the image.
__device__ __forceinline__ void chk_img(const Img& im, int row, int col) {
  FOBF_CHK(im,
           row >= 0 && row < im.H && col >= 0 && col < im.W && col < im.ld_in,
           FOBF_CHECK_IMAGE);
}

// n floats at p lie inside the workspace (workspace forms) or the LDS
// allocation (N and D in LDS).
__device__ __forceinline__ void chk_nd(const Img& im, const float* p, int n) {
#if FOBF_CHECKS
  if (im.ws)
    FOBF_CHK(im, p >= im.ws && p + n <= im.ws + im.ws_floats, FOBF_CHECK_WS);
  else
    chk_lds(im, p, 4 * n);
#endif
}

// A non-zero horizontal tap w joins window column c (counted from the
// first column of the strip's window, x0w - r) to output column n of the
// strip only within the output's window: 0 <= c - n <= 2r.
__device__ __forceinline__ void chk_htap(const Img& im, float w, int c, int n) {
  FOBF_CHK(im, w == 0.f || (c - n >= 0 && c - n <= 2 * im.r), FOBF_CHECK_HALO_H);
}
// the same for a vertical tap joining ring row h (counted from the first
// row of the output block's window) to output row m of the block
__device__ __forceinline__ void chk_vtap(const Img& im, float w, int h, int m) {
  FOBF_CHK(im, w == 0.f || (h - m >= 0 && h - m <= 2 * im.r), FOBF_CHECK_HALO_V);
}

// The float32 Toeplitz slices as every reader indexes them (lane's Bt[s]
// for window column SH (lane/16) + s, At[4d + v] for ring row 16 d + 4 v
// + lane/16, against output column / row lane%16): in the LDS, and
// non-zero only inside the windows.  Once per channel group: the readers
// index them the same way for every block.
template <int SH>
__device__ __forceinline__ void chk_f32_tables(const Img& im, const float* Bt, const float* At,
                                               int lane) {
#if FOBF_CHECKS
  constexpr int DV = (SH + 3) / 4;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll 1
  for (int s = 0; s < 4 * DV; ++s) {
    chk_lds(im, Bt + s * 64 + lane, 4);
    chk_lds(im, At + s * 64 + lane, 4);
    if (s < SH) chk_htap(im, Bt[s * 64 + lane], SH * lk + s, li);
    chk_vtap(im, At[s * 64 + lane], 4 * s + lk, li);
    // the vertical steps skipped (s >= SH) must carry only zero taps
    FOBF_CHK(im, s < SH || At[s * 64 + lane] == 0.f, FOBF_CHECK_HALO_V);
  }
#endif
}

// Which horizontal block each slot of a vertical ring holds (check builds
// only): the vertical pass of output block pb must find block pb + d in
// the slot it takes for its d-th block.
template <int DV>
struct RingTags {
#if FOBF_CHECKS
  int q[DV];
  __device__ __forceinline__ void set(int u, int v) { q[u] = v; }
  __device__ __forceinline__ void check(const Img& im, int slot, int want) const {
    FOBF_CHK(im, q[slot] == want, FOBF_CHECK_RING);
  }
#else
  __device__ __forceinline__ void set(int, int) {}
  __device__ __forceinline__ void check(const Img&, int, int) const {}
#endif
};

// Fills the launch's dynamic LDS with all-ones words (NaN in float32, fp16
// and bf16) from `from_bytes` on, then waits for the workgroup: a later
// read of a word the kernel never wrote carries NaN into the output.
__device__ __forceinline__ void poison_lds(const Img& im, int from_bytes = 0) {
#if FOBF_CHECKS
  extern __shared__ float fobf_dyn_lds[];
  uint32_t* w = reinterpret_cast<uint32_t*>(fobf_dyn_lds);
  for (int i = from_bytes / 4 + static_cast<int>(threadIdx.x); i < im.lds_bytes / 4;
       i += blockDim.x)
    w[i] = 0xffffffffu;
  __syncthreads();
#endif
}

// Copies the image's tables into LDS.  A macro, not a function: the kernel
// parameter block must be indexed in the kernel body itself (taking its
// address for a callee would copy it to scratch memory).
#define FOBF_LOAD_TABLES(p, tbl)                                              \
  do {                                                                        \
    for (int m_ = threadIdx.x; m_ <= (p).r; m_ += blockDim.x) (tbl)[m_] = (p).g[m_];    \
    for (int k_ = threadIdx.x; k_ < (p).K; k_ += blockDim.x)                             \
      (tbl)[64 + k_] = (p).c_dev ? (p).c_dev[k_] : (p).c[k_];                 \
    for (int j_ = threadIdx.x; j_ <= 2 * (p).r + 1; j_ += blockDim.x)                   \
      (tbl)[96 + j_] = (p).gsum[j_];                                          \
  } while (0)

// =========================================================================
// float32: 16x16x4 MFMA, channels on the fly, N/D in LDS
// =========================================================================

// Block row whose channels lane li feeds to the horizontal product (its A
// row li): rows 4 (li % 4) + li / 4, a transposition of the 4 x 4 row
// index.  The product's result register v of lane l (result row 4 (l/16)
// + v) then holds block row 4 v + l/16, so the vertical step that takes
// register v contracts the four consecutive rows 4v .. 4v + 3 of a block
// instead of rows v, v + 4, v + 8, v + 12.  Vertical step j = 4 d + v then
// meets non-zero taps only while 4 j <= 15 + 2r, i.e. for j < SH: the
// steps from SH to 4 DV - 1 (all-zero Toeplitz slices) are skipped.
__device__ __forceinline__ int hrow_of_lane(int li) { return 4 * (li & 3) + (li >> 2); }

// One channel group over this wave's strip: G = 1 is {f} (k = 0, no trig),
// G = 4 is {C f, S f, C, S} of frequency k >= 1, G = 5 is f followed by
// frequency k = 1's four channels (the f channel's single accumulator
// chain then overlaps four others; its fold adds f's term and then
// frequency 1's, the order of two separate passes, so the output is the
// same bit for bit).  Bt / At are the
// horizontal / vertical Toeplitz slices, one float per lane per MFMA step,
// precomputed in LDS.
//
// SH = ceil((16 + 2r) / 4) horizontal 4-column steps is a template
// parameter, so that the step loop has no branches and the compiler can
// overlap one step's trig with the previous step's matrix work.
//
// EDGE = false is the interior path: every pixel the strip touches lies in
// the image, so loads need no clamping (one address per row, immediate
// offsets) and channels no masks.  On gfx950 the fp32 matrix instruction
// does not overlap vector-ALU work, so every vector instruction removed
// from the step loop is time saved.  EDGE = true clamps loads and zeroes
// the channels of out-of-image neighbours.
//
// The contraction index of a horizontal step does not have to run over
// adjacent columns: step s takes column c = SH*kk + s of the strip's window
// (kk = lane / 16, the MFMA's k index), and the Toeplitz slice Bt is built
// for that order.  Each lane then reads SH adjacent floats of one row, a
// few wide loads per block instead of one 4-byte load per step.
//
// The image values of the next 16-row block are loaded during the current
// block's steps: each value is replaced by its successor right after its
// last use, so the load has a whole block of matrix work to land.
template <int SH, int G, bool EDGE>
__device__ __forceinline__ void f32_group(const Img& im, int k, int x0w, int y0,
                                          int nblk, const float* tbl, const float* Bt,
                                          const float* At, float* Ns, float* Ds, int lane) {
  constexpr int DV = (SH + 3) / 4;            // H blocks per vertical block
  const float* cS = tbl + 64;
  const int r = im.r;
  const int li = lane & 15;
  const int lk = lane >> 4;
  const int hr = hrow_of_lane(li);   // block row of this lane's A operand
  const float kinv = static_cast<float>(k) * im.inv_period;
  const float ck = cS[k];
  const int QB = nblk + DV - 1;
  const int colbase = x0w - r + SH * lk;
  const int gxo = min(x0w + li, im.W - 1);
  const size_t ld = static_cast<size_t>(im.ld_in);

  // address of (row y0 - r + 16 q + hr, column colbase) -- interior only
  auto rowptr = [&](int q) { return im.in + (y0 - r + 16 * q + hr) * ld + colbase; };
  auto load_block = [&](int q, float (&v)[SH]) {
    if (!EDGE) {
      const float* p = rowptr(q);
      chk_img(im, y0 - r + 16 * q + hr, colbase);
      chk_img(im, y0 - r + 16 * q + hr, colbase + SH - 1);
#pragma unroll
      for (int s = 0; s < SH; ++s) v[s] = p[s];
    } else {
      const int row = y0 - r + 16 * q + hr;
      const float* rp = im.in + static_cast<size_t>(min(max(row, 0), im.H - 1)) * ld;
#pragma unroll
      for (int s = 0; s < SH; ++s) v[s] = rp[min(max(colbase + s, 0), im.W - 1)];
    }
  };

  f4 ring[DV][G];
  RingTags<DV> tags;
  chk_f32_tables<SH>(im, Bt, At, lane);
  float fv[SH];
  load_block(0, fv);

  for (int qq = 0; qq < QB; qq += DV) {
#pragma unroll
    for (int u = 0; u < DV; ++u) {
      const int q = qq + u;
      if (q < QB) {
        const int pb = q - (DV - 1);
        // output-pixel values for this block's fold, issued first so that
        // they land during the block's matrix work (rows clamped: blocks
        // with pb < 0 fold nothing); the scheduling group keeps the loads
        // at the head of the block
        float fo[4];
        if (G >= 4) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int gy = min(max(y0 + 16 * pb + 4 * lk + v, 0), im.H - 1);
            chk_img(im, gy, gxo);
            fo[v] = im.in[gy * ld + gxo];
          }
          __builtin_amdgcn_sched_group_barrier(0x020, 4, 0);
        }
        // next block's row (the last block reloads its own row: branch-free)
        const int qn = (q + 1 < QB) ? q + 1 : q;
        const int rown = y0 - r + 16 * qn + hr;
        const float* pn = EDGE ? im.in + static_cast<size_t>(min(max(rown, 0), im.H - 1)) * ld
                               : rowptr(qn);
        if (!EDGE) {
          chk_img(im, rown, colbase);
          chk_img(im, rown, colbase + SH - 1);
        }
        // ---- horizontal pass, H rows 16q .. 16q+15 of the strip ----
        const int row = y0 - r + 16 * q + hr;
        const bool rin = !EDGE || static_cast<unsigned>(row) < static_cast<unsigned>(im.H);
        f4 acc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < SH; ++s) {
          float f = fv[s];
          float m = 1.f;
          if (EDGE) {
            const bool in = rin && static_cast<unsigned>(colbase + s) <
                                       static_cast<unsigned>(im.W);
            f = in ? f : 0.f;
            m = in ? 1.f : 0.f;
          }
          fv[s] = EDGE ? pn[min(max(colbase + s, 0), im.W - 1)] : pn[s];
          const float bh = Bt[s * 64 + lane];
          float a[G];
          if (G == 1) {
            a[0] = f;
          } else {
            constexpr int g0 = G == 5 ? 1 : 0;
            float sn, cs;
            sincos_rev(kinv * f, &sn, &cs);
            if (G == 5) a[0] = f;
            a[g0] = cs * f;
            a[g0 + 1] = sn * f;
            a[g0 + 2] = EDGE ? cs * m : cs;
            a[g0 + 3] = EDGE ? sn * m : sn;
          }
#pragma unroll
          for (int g = 0; g < G; ++g)
            acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[g], bh, acc[g], 0, 0, 0);
        }
#pragma unroll
        for (int g = 0; g < G; ++g) ring[u][g] = acc[g];
        tags.set(u, q);

        // ---- vertical pass, output block pb ----
        if (pb >= 0) {
          f4 vacc[G];
#pragma unroll
          for (int g = 0; g < G; ++g) vacc[g] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int d = 0; d < DV; ++d) {
            const int slot = (u + 1 + d) % DV;
            tags.check(im, slot, pb + d);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              if (4 * d + v >= SH) break;   // all-zero slices
              const float av = At[(d * 4 + v) * 64 + lane];
#pragma unroll
              for (int g = 0; g < G; ++g)
                vacc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, ring[slot][g][v], vacc[g],
                                                               0, 0, 0);
            }
          }
          // ---- fold into N, D with the output pixel's own trig ----
          // (all reads of N, D first: they may alias the writes, so reads
          // issued after a write would each wait for the LDS round trip)
          float* const nrow = Ns + pb * 256 + lane;
          float* const drow = Ds + pb * 256 + lane;
          float nv[4], dv[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            nv[v] = nrow[64 * v];
            if (G >= 4) dv[v] = drow[64 * v];
          }
          chk_nd(im, nrow, 193);
          chk_nd(im, drow, 193);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if (G == 1) {
              nv[v] = fmaf(ck, vacc[0][v], nv[v]);
            } else {
              constexpr int g0 = G == 5 ? 1 : 0;
              if (G == 5) nv[v] = fmaf(cS[0], vacc[0][v], nv[v]);
              float sn, cs;
              sincos_rev(kinv * fo[v], &sn, &cs);
              nv[v] = fmaf(ck, fmaf(cs, vacc[g0][v], sn * vacc[g0 + 1][v]), nv[v]);
              dv[v] = fmaf(ck, fmaf(cs, vacc[g0 + 2][v], sn * vacc[g0 + 3][v]), dv[v]);
            }
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            nrow[64 * v] = nv[v];
            if (G >= 4) drow[64 * v] = dv[v];
          }
        }
      }
    }
  }
}

// True when every pixel a strip's horizontal pass and fold touch lies in
// the image (no clamping or masking needed).
template <int SH>
__device__ __forceinline__ bool strip_interior(const Img& im, int x0w, int y0, int nblk) {
  constexpr int DV = (SH + 3) / 4;
  const int r = im.r;
  return x0w - r >= 0 && x0w - r + 4 * SH <= im.W && y0 - r >= 0 &&
         y0 - r + 16 * (nblk + DV - 1) <= im.H;
}

// Per-lane N and D of the wave's strip live in LDS at ((pb*4 + v)*64 +
// lane) for output pixel (row 16 pb + 4 (lane/16) + v, column lane % 16):
// one 16-row block is 256 consecutive floats, so a wave's access is
// bank-conflict free.
// N = 0, D = c_0 W(i).
__device__ __forceinline__ void init_nd(const Img& im, const float* tbl, int x0w, int y0,
                                        int nblk, float* Ns, float* Ds, int lane) {
  const float* cS = tbl + 64;
  const float* sS = tbl + 96;
  const float wx = edge_weight(sS, x0w + (lane & 15), im.W, im.r);
  for (int pb = 0; pb < nblk; ++pb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float wy = edge_weight(sS, y0 + 16 * pb + 4 * (lane >> 4) + v, im.H, im.r);
      const int idx = (pb * 4 + v) * 64 + lane;
      chk_nd(im, Ns + idx, 1);
      chk_nd(im, Ds + idx, 1);
      Ns[idx] = 0.f;
      Ds[idx] = cS[0] * wx * wy;
    }
}

__device__ __forceinline__ void store_nd(const Img& im, int x0w, int y0, int nblk,
                                         const float* Ns, const float* Ds, int lane,
                                         float shift = 0.f) {
  const int gx = x0w + (lane & 15);
  for (int pb = 0; pb < nblk; ++pb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gy = y0 + 16 * pb + 4 * (lane >> 4) + v;
      const int idx = (pb * 4 + v) * 64 + lane;
      if (gy < im.H && gx < im.W) {
        chk_nd(im, Ns + idx, 1);
        chk_nd(im, Ds + idx, 1);
        FOBF_CHK(im, gy >= 0 && gx >= 0 && gx < im.ld_out, FOBF_CHECK_OUT);
        im.out[static_cast<size_t>(gy) * im.ld_out + gx] = Ns[idx] / Ds[idx] + shift;
      }
    }
}

// Toeplitz slices as per-lane LDS tables: Bt[s][lane] (horizontal step s,
// window column SH*(lane/16) + s against output column lane%16; 4*DV
// entries, those beyond SH unused) and At[j][lane] (vertical step j = 4d +
// v: ring block d, rows 4v + lane/16, see hrow_of_lane; 4*DV entries, those
// from SH on all zero and skipped).
template <int SH>
__device__ __forceinline__ void build_f32_tables(const Img& im, const float* gS, int r, float* Bt,
                                                 float* At) {
  constexpr int DV = (SH + 3) / 4;
  for (int i = threadIdx.x; i < 4 * DV * 64; i += blockDim.x) {
    const int s = i >> 6, l = i & 63;
    chk_lds(im, Bt + i, 4);
    chk_lds(im, At + i, 4);
    Bt[i] = tap(gS, SH * (l >> 4) + s - r - (l & 15), r);
    At[i] = tap(gS, 4 * s + (l >> 4) - r - (l & 15), r);
  }
}

// XCD-aware tile order.  Workgroups are dealt to the 8 XCDs round-robin
// (block L runs on XCD L % 8); each XCD is given a contiguous run of tiles,
// walked in panels 8 tiles wide, so the tiles resident on one XCD share
// their halos in that XCD's L2.  Returns false for padding blocks.
__device__ __forceinline__ bool tile_of_block(int L, int nblocks, int ntx, int nty, int* tx,
                                              int* ty) {
  const int per = nblocks >> 3;
  const int t = (L & 7) * per + (L >> 3);
  if (t >= ntx * nty) return false;
  constexpr int PW = 8;
  const int panel = t / (PW * nty);
  const int rem = t - panel * PW * nty;
  const int pw = min(PW, ntx - panel * PW);
  *ty = rem / pw;
  *tx = panel * PW + (rem - *ty * pw);
  return true;
}

// MERGE: f is taken with frequency 1 (G = 5, same output as separate
// passes; the single-image and batch kernels take it at no register cost).
template <int SH, bool MERGE = false>
__device__ __forceinline__ void f32_tile(const Img& im, int tx, int ty, int nblk,
                                         const float* tbl, const float* Bt, const float* At,
                                         float* nd) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  float* Ns = nd + wave * 2 * nblk * 256;
  float* Ds = Ns + nblk * 256;
  const int x0w = tx * (MWAVES * MSTRIP) + wave * MSTRIP;
  const int y0 = ty * 16 * nblk;
  init_nd(im, tbl, x0w, y0, nblk, Ns, Ds, lane);
  const bool merge = MERGE && im.K > 1;
  const int k1 = merge ? 2 : 1;
  if (strip_interior<SH>(im, x0w, y0, nblk)) {
    if (merge)
      f32_group<SH, 5, false>(im, 1, x0w, y0, nblk, tbl, Bt, At, Ns, Ds, lane);
    else
      f32_group<SH, 1, false>(im, 0, x0w, y0, nblk, tbl, Bt, At, Ns, Ds, lane);
    for (int k = k1; k < im.K; ++k)
      f32_group<SH, 4, false>(im, k, x0w, y0, nblk, tbl, Bt, At, Ns, Ds, lane);
  } else {
    if (merge)
      f32_group<SH, 5, true>(im, 1, x0w, y0, nblk, tbl, Bt, At, Ns, Ds, lane);
    else
      f32_group<SH, 1, true>(im, 0, x0w, y0, nblk, tbl, Bt, At, Ns, Ds, lane);
    for (int k = k1; k < im.K; ++k)
      f32_group<SH, 4, true>(im, k, x0w, y0, nblk, tbl, Bt, At, Ns, Ds, lane);
  }
  store_nd(im, x0w, y0, nblk, Ns, Ds, lane);
}


// =========================================================================
// staged fp16 / bf16: 16x16x32 MFMA, channels shared through LDS, N/D in
// LDS
// =========================================================================

template <typename OT>
struct Stage;

template <>
struct Stage<_Float16> {
  typedef _Float16 T;                     // staged word
  typedef h8 v8;
  static constexpr int kParts = 1;        // one fp16 word per staged value
  __device__ static __forceinline__ f4 mfma(v8 a, v8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  // K = 16 product: one horizontal block (4 words per lane) per operand
  __device__ static __forceinline__ f4 mfma16(h4 a, h4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ _Float16 cvt(float x) { return static_cast<_Float16>(x); }
  // two staged values as one 32-bit word (round to nearest)
  __device__ static __forceinline__ void pack2(float x0, float x1, uint32_t (&w)[1]) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const h2 v = {static_cast<_Float16>(x0), static_cast<_Float16>(x1)};
    w[0] = __builtin_bit_cast(uint32_t, v);
  }
};

template <>
struct Stage<__bf16> {
  typedef __bf16 T;
  typedef b8 v8;
  // bf16 keeps 8 mantissa bits (relative rounding 2^-9).  The output
  // divides N by D, and where D/W is small (a pixel unlike most of its
  // window) that rounding is amplified past half an intensity level.  Every
  // staged value -- channel, tap and horizontal result -- is therefore held
  // as hi + lo bf16 words (v = hi + lo, |lo| <= 2^-9 |v|) and each product
  // is formed as hi*hi + hi*lo + lo*hi, leaving ~2^-16 relative error.
  static constexpr int kParts = 2;
  __device__ static __forceinline__ f4 mfma(v8 a, v8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ f4 mfma16(bh4 a, bh4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, a),
                                                     __builtin_bit_cast(s4, b), c, 0, 0, 0);
  }
  __device__ static __forceinline__ __bf16 cvt(float x) { return static_cast<__bf16>(x); }
  // two staged values as hi and lo words.  For the staged channels hi is
  // the truncation of x (its upper 16 bits, one byte permute for the pair)
  // and lo the remainder x - hi (exact in float32) rounded to bf16: the
  // pair still carries x to ~2^-17 relative, with fewer conversions than
  // rounding hi first.
  // (remainders subtracted as written: never fused with the product that
  // made x, so every build of the kernel splits a value the same way)
  __device__ static __forceinline__ void pack2(float x0, float x1, uint32_t (&w)[2]) {
#pragma clang fp contract(off)
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    const uint32_t u0 = __builtin_bit_cast(uint32_t, x0);
    const uint32_t u1 = __builtin_bit_cast(uint32_t, x1);
    w[0] = __builtin_amdgcn_perm(u1, u0, 0x07060302u);   // upper halves of u0, u1
    const float r0 = x0 - __builtin_bit_cast(float, u0 & 0xffff0000u);
    const float r1 = x1 - __builtin_bit_cast(float, u1 & 0xffff0000u);
    const b2 v = {static_cast<__bf16>(r0), static_cast<__bf16>(r1)};
    w[1] = __builtin_bit_cast(uint32_t, v);
  }
};

// Two-word fp16 staging: every staged value, tap and horizontal result is
// held as hi + lo fp16 words (hi rounded to nearest, lo the rounded
// remainder: v = hi + lo to ~2^-22 relative) and products are hi*hi +
// hi*lo + lo*hi on the fp16 matrix cores -- float32-class accuracy from
// the staged kernel.  The tag selects this mode; the words are _Float16.
struct F16Pair {};

template <>
struct Stage<F16Pair> {
  typedef _Float16 T;
  typedef h8 v8;
  static constexpr int kParts = 2;
  __device__ static __forceinline__ f4 mfma(v8 a, v8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ f4 mfma16(h4 a, h4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ _Float16 cvt(float x) { return static_cast<_Float16>(x); }
  __device__ static __forceinline__ void pack2(float x0, float x1, uint32_t (&w)[2]) {
#pragma clang fp contract(off)
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const h2 hi = {static_cast<_Float16>(x0), static_cast<_Float16>(x1)};
    const h2 lo = {static_cast<_Float16>(x0 - static_cast<float>(hi[0])),
                   static_cast<_Float16>(x1 - static_cast<float>(hi[1]))};
    w[0] = __builtin_bit_cast(uint32_t, hi);
    w[1] = __builtin_bit_cast(uint32_t, lo);
  }
};

// LDS pitch (elements) of a staged channel row: >= cw, = 16 (mod 64).  Of
// the residues 8, 16, 24, 40 and 56 (all keep the 16-byte reads aligned)
// 16 is the fastest for every staged kernel at 4096^2, theta = 10 (3-4%
// over 24), and the only one that clears the LDS bank-conflict counter
// (0 cycles; 8 and 24 read 1.4x the LDS instruction cycles in conflicts,
// 4 per 16-byte read).
__host__ __device__ constexpr int stage_pitch(int cw) { return ((cw + 47) / 64) * 64 + 16; }
// staged columns: the window of the last of NW strips ends at
// 16 (NW - 1) + 32 SHS (columns past 16 NW + 2r only ever meet zero taps)
__host__ __device__ constexpr int stage_cols(int shs, int nw) { return 16 * (nw - 1) + 32 * shs; }
constexpr int STAGE_CH = 4;   // channels per staged buffer (per word part)

// Channel groups of one pass over a tile.  A group is {f} (k = 0, no trig),
// one frequency k (C_k f, S_k f, C_k, S_k), f with frequency 1 (5 channels)
// or two frequencies k, k+1 (8 channels): G = [f] + 4 NF.  The workspace
// form of single-word fp16 merges groups that way, so that N and D make 4
// instead of 8 round trips through the workspace at K = 8 and the fold's
// pixel values are fetched once per two frequencies; it then stages eight
// channels per buffer.  Each channel's products and each pixel's sequence
// of additions into N and D are those of one-frequency groups, so the
// output is unchanged bit for bit.  The other forms stage four channels.
template <int G>
constexpr bool group_has_f() { return G % 4 == 1; }
template <int G>
constexpr int group_freqs() { return G / 4; }
template <typename OT, bool GND>
constexpr bool staged_merge() { return GND && Stage<OT>::kParts == 1; }
// The two-word workspace forms take f with frequency 1 (five channels) at
// DV <= 4; their horizontal Toeplitz slices then live in the LDS, which
// frees the registers the fifth channel's ring takes.  Same output bit for
// bit; measured at 4096^2, K = 8: -2 to -4% at theta = 2.5, 5, 8, and +1.5%
// at DV = 5 (theta = 10), where it is not used.
template <typename OT, int DV, bool GND>
constexpr bool staged_fmerge2() { return GND && Stage<OT>::kParts == 2 && DV <= 4; }
template <typename OT, int DV, bool GND>
constexpr int staged_channels() {
  return staged_merge<OT, GND>() ? 8 : (staged_fmerge2<OT, DV, GND>() ? 5 : STAGE_CH);
}

// Staging items: IW consecutive columns of one row of a 16-row block, one
// item per thread.  Only the CWn = 16 NW + 2r columns that meet non-zero
// taps are built (the tail stays as zeroed at tile start).  With r <= 8 (DV
// - 1), a block has at most 16 (16 NW + 16 (DV - 1)) such pixels; IW is the
// smallest even width that spreads them over the 64 NW threads, so that
// every wave takes an equal share of the staging work.
template <int DV, int NW>
constexpr int stage_item_width() { return 2 * ((2 * (NW + DV - 1) + NW - 1) / NW); }

// Staged row width: the columns the horizontal steps read, and those the
// staging items cover.
template <int DV, int NW>
constexpr int stage_width() {
  return stage_cols((DV + 1) / 2, NW) > 16 * NW + 16 * (DV - 1) + stage_item_width<DV, NW>()
             ? stage_cols((DV + 1) / 2, NW)
             : 16 * NW + 16 * (DV - 1) + stage_item_width<DV, NW>();
}

// Staging buffers per workgroup: two would let a block be staged while the
// one before it is still being read (one barrier per block); one buffer
// costs a second barrier per block but halves the staging LDS, which pays
// for taller tiles (less vertical halo) and wider workgroups: measured at
// 4096^2, r = 30, fp16 0.75 -> 0.62 ms and bf16 1.61 -> 1.28 ms.  The
// workspace form (GND: N and D outside the LDS) has the room for two, and
// there they save 1-3%.
template <typename OT, int NW, bool GND = false>
constexpr int staged_bufs() { return GND ? 2 : 1; }

// The staging region: the channel buffers, then (two-word modes at eight
// strips only) the per-lane vertical Toeplitz slices, which would otherwise
// hold 24 VGPRs per lane through the whole group at the kernel's register
// limit.  Four-strip workgroups (the batch kernel) keep them in registers:
// there the LDS is worth more as tile height.
template <typename OT, int DV, int NW, bool GND = false>
constexpr size_t staged_stage_bytes() {
  return sizeof(typename Stage<OT>::T) * staged_bufs<OT, NW, GND>() * Stage<OT>::kParts *
         staged_channels<OT, DV, GND>() * 16 * stage_pitch(stage_width<DV, NW>());
}

template <typename OT, int NW>
constexpr bool staged_vtap_in_lds() { return Stage<OT>::kParts == 2 && NW == 8; }

template <typename OT, int DV, int NW>
constexpr size_t staged_vtap_bytes() {
  return staged_vtap_in_lds<OT, NW>() ? static_cast<size_t>((DV + 1) / 2) * 2 * 64 * 16 : 0;
}

template <typename OT, int DV, int NW, bool GND = false>
constexpr size_t staged_htap_bytes() {
  return staged_fmerge2<OT, DV, GND>() ? static_cast<size_t>((DV + 1) / 2) * 2 * 64 * 16 : 0;
}

template <typename OT, int DV, int NW, bool GND = false>
constexpr size_t staged_buf_bytes() {
  return staged_stage_bytes<OT, DV, NW, GND>() + staged_vtap_bytes<OT, DV, NW>() +
         staged_htap_bytes<OT, DV, NW, GND>();
}

// Issues the global loads of this thread's item of one block into
// registers.  Called one block ahead of stage_block, so that the loads land
// during the matrix work of the current block instead of stalling the
// staging.  Loads are clamped into the image; stage_block zeroes what lies
// outside.
template <int IW>
__device__ __forceinline__ void stage_fetch(const Img& im, int x0, int row0, int CWn,
                                            bool interior, float (&fv)[IW]) {
  const int per_row = (CWn + IW - 1) / IW;
  const int it = threadIdx.x;
  if (it >= 16 * per_row) return;
  const int rr = it / per_row;
  const int row = row0 + rr;
  const int col0 = x0 - im.r + (it - rr * per_row) * IW;
  if (interior) {
    const float* p = im.in + static_cast<size_t>(row) * im.ld_in + col0;
    chk_img(im, row, col0);
    chk_img(im, row, col0 + IW - 1);
#pragma unroll
    for (int j = 0; j < IW; ++j) fv[j] = p[j];
  } else {
    const float* rp = im.in + static_cast<size_t>(min(max(row, 0), im.H - 1)) * im.ld_in;
#pragma unroll
    for (int j = 0; j < IW; ++j) fv[j] = rp[min(max(col0 + j, 0), im.W - 1)];
  }
}

// Builds this thread's item of one 16-row block of a group of G channels
// (frequencies k, k+1, .. as group_freqs; f first when group_has_f) into
// LDS from the values stage_fetch loaded.  Element (row, col) of channel g,
// word part h sits at buf[((h * SCH + g) * 16 + row) * PC + col], col 0 =
// column x0 - r.  `interior`: the block's items lie inside the image (no
// masks).
template <typename OT, int G, int IW, bool INTERIOR, int SCH = STAGE_CH>
__device__ __forceinline__ void stage_block(const Img& im, int k, float shift, int x0,
                                           int row0, int CWn, int PC, typename Stage<OT>::T* buf,
                                           const float (&fvs)[IW]) {
  constexpr bool HF = group_has_f<G>();
  constexpr int NF = group_freqs<G>();
  static_assert(G == (HF ? 1 : 0) + 4 * NF && G <= SCH, "bad channel group");
  using S = Stage<OT>;
  constexpr int NP = S::kParts;
  const int per_row = (CWn + IW - 1) / IW;
  const int it = threadIdx.x;
  if (it >= 16 * per_row) return;
  const int rr = it / per_row;
  const int c0 = (it - rr * per_row) * IW;
  const int row = row0 + rr;
  const int col0 = x0 - im.r + c0;
  const bool rin = static_cast<unsigned>(row) < static_cast<unsigned>(im.H);
  bool in[IW];
  float fs[IW];
#pragma unroll
  for (int j = 0; j < IW; ++j) {
    in[j] = INTERIOR || (rin && static_cast<unsigned>(col0 + j) < static_cast<unsigned>(im.W));
    fs[j] = in[j] ? fvs[j] - shift : 0.f;     // f - m, zero outside
  }
  // IW is even and c0 a multiple of IW: pairs of words are 4-byte aligned
  FOBF_CHK(im, rr < 16 && c0 + IW <= PC, FOBF_CHECK_STAGE);
  auto put = [&](int g, const float (&x)[IW]) {
    chk_lds(im, buf + (g * 16 + rr) * PC + c0, IW * sizeof(typename S::T));
    chk_lds(im, buf + (((NP - 1) * SCH + g) * 16 + rr) * PC + c0, IW * sizeof(typename S::T));
#pragma unroll
    for (int j = 0; j < IW / 2; ++j) {
      uint32_t w[NP];
      S::pack2(x[2 * j], x[2 * j + 1], w);
#pragma unroll
      for (int h = 0; h < NP; ++h)
        reinterpret_cast<uint32_t*>(buf + ((h * SCH + g) * 16 + rr) * PC + c0)[j] = w[h];
    }
  };
  if (HF) put(0, fs);
  // one frequency at a time: its four channels are written before the
  // next frequency's trig, which bounds the registers a group needs
#pragma unroll
  for (int q = 0; q < NF; ++q) {
    constexpr int g0 = HF ? 1 : 0;
    const float kinv = static_cast<float>(k + q) * im.inv_period;
    float x[4][IW];
#pragma unroll
    for (int j = 0; j < IW; ++j) {
      const float f = in[j] ? fvs[j] : 0.f;
      float sn, cs;
      sincos_rev(kinv * f, &sn, &cs);
      x[0][j] = cs * fs[j];
      x[1][j] = sn * fs[j];
      x[2][j] = in[j] ? cs : 0.f;
      x[3][j] = in[j] ? sn : 0.f;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) put(g0 + 4 * q + c, x[c]);
  }
}

// =========================================================================
// float32, workspace form: the channels of each 16-row block staged once
// per workgroup in LDS (float32), N and D in the global workspace
// =========================================================================

// LDS pitch (floats) of a staged float32 channel row: room for the items
// (CWn rounded up to whole items) and the strips' reads, = 2 (mod 32): each
// half-wave of a read (16 rows x 2 column runs SH apart) then falls in 32
// distinct banks (measured 0.2-1.5% faster than a pitch = 4 (mod 64)).
__host__ __device__ constexpr int f32s_pitch(int sh, int nw, int r, int iw) {
  const int a = 16 * nw + 2 * r + iw, b = 16 * (nw - 1) + 4 * sh;
  const int m = a > b ? a : b;
  return ((m - 2 + 31) / 32) * 32 + 2;
}

// Channels per staging buffer of the float32 workspace form: its first
// pass takes f together with frequency 1 (five channels), so that the f
// channel's products (one accumulator chain on its own) overlap four
// others and N and D make one round trip fewer; the sums and the order of
// the additions into N and D are those of separate passes.
constexpr int kF32Ch = 5;

// This thread's item of one block: a group of G channels (f alone, one
// frequency k: C f, S f, C, S, or f then frequency k) (float32, no shift)
// into buf[(g * 16 + row) * PC + col], col 0 = column x0 - r.
template <int G, int IW, bool INTERIOR>
__device__ __forceinline__ void f32s_stage(const Img& im, float kinv, int x0, int row0, int CWn,
                                           int PC, float* buf, const float (&fvs)[IW]) {
  constexpr bool HF = group_has_f<G>();
  constexpr int g0 = HF ? 1 : 0;
  const int per_row = (CWn + IW - 1) / IW;
  const int it = threadIdx.x;
  if (it >= 16 * per_row) return;
  const int rr = it / per_row;
  const int c0 = (it - rr * per_row) * IW;
  const int row = row0 + rr;
  const int col0 = x0 - im.r + c0;
  const bool rin = static_cast<unsigned>(row) < static_cast<unsigned>(im.H);
  float x[G][IW];
#pragma unroll
  for (int j = 0; j < IW; ++j) {
    const bool in =
        INTERIOR || (rin && static_cast<unsigned>(col0 + j) < static_cast<unsigned>(im.W));
    const float f = in ? fvs[j] : 0.f;
    if (HF) x[0][j] = f;
    if (G >= 4) {
      float sn, cs;
      sincos_rev(kinv * f, &sn, &cs);
      x[g0][j] = cs * f;
      x[g0 + 1][j] = sn * f;
      x[g0 + 2][j] = in ? cs : 0.f;
      x[g0 + 3][j] = in ? sn : 0.f;
    }
  }
  // IW is even and c0 a multiple of it: pairs are 8-byte aligned (the row
  // pointer pinned: the writes then take their offsets in the instruction)
  FOBF_CHK(im, rr < 16 && c0 + IW <= PC, FOBF_CHECK_STAGE);
  chk_lds(im, buf + rr * PC + c0, 4 * IW);
  chk_lds(im, buf + ((G - 1) * 16 + rr) * PC + c0, 4 * IW);
  float* const wrow = lds_pinned(buf + rr * PC + c0);
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int j = 0; j < IW / 2; ++j)
      reinterpret_cast<float2*>(wrow + g * 16 * PC)[j] = float2{x[g][2 * j], x[g][2 * j + 1]};
}

// One channel group over the workgroup's tile: per 16-row block the
// workgroup stages the block's channels (two buffers, one barrier per
// block), each wave runs the horizontal pass of its strip from LDS (the
// contraction order of f32_group: lane (li, lk), step s reads column
// 16 wave + SH lk + s), the vertical pass from its ring and folds into the
// block's N and D, fetched from the workspace a block ahead.  TREG: the
// lane's Toeplitz slices are held in registers (btr, atr) instead of being
// read from LDS per step (1% at r <= 30, where the registers are free).
template <int SH, int NW, int G, bool TREG>
__device__ __forceinline__ void f32s_group(const Img& im, int k, int x0, int y0, int nblk,
                                           const float* tbl, const float* Bt, const float* At,
                                           float* sbuf, int PC, float* Ns, float* Ds,
                                           const float (&btr)[SH],
                                           const float (&atr)[4 * ((SH + 3) / 4)]) {
  constexpr int DV = (SH + 3) / 4;
  constexpr int IW = stage_item_width<DV, NW>();
  constexpr bool HF = group_has_f<G>();      // f first (c_0 into N)
  constexpr bool HK = G >= 4;                // frequency k (channels from g0)
  constexpr int g0 = HF ? 1 : 0;
  static_assert(G == 1 || G == 4 || G == 5, "bad channel group");
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const float kinv = static_cast<float>(k) * im.inv_period;
  const float ck = tbl[64 + k];
  const float c0 = tbl[64];
  const int r = im.r;
  const int CWn = 16 * NW + 2 * r;
  const int x0w = x0 + wave * MSTRIP;
  const int gxo = min(x0w + li, im.W - 1);
  const int QB = nblk + DV - 1;
  const bool cols_in = x0 - r >= 0 && x0 - r + IW * ((CWn + IW - 1) / IW) <= im.W;
  auto block_interior = [&](int row0) { return cols_in && row0 >= 0 && row0 + 16 <= im.H; };
  const size_t ld = static_cast<size_t>(im.ld_in);
  // the fold's pixel values: where every output row of the tile lies in
  // the image, block pb's four rows are at a fixed stride from one base
  // (blocks with pb < 0 fold nothing: they read block 0's)
  const bool rows_in = y0 + 16 * nblk <= im.H;
  const float* const fo_base = im.in + static_cast<size_t>(min(y0 + 4 * lk, im.H - 1)) * ld + gxo;

  f4 ring[DV][G];
  RingTags<DV> tags;
  // (check builds) the slices, and the last column a lane's steps read
  chk_f32_tables<SH>(im, Bt, At, lane);
  FOBF_CHK(im, 16 * wave + SH * lk + SH <= PC, FOBF_CHECK_HALO_H);
  float fvs[IW];
  stage_fetch<IW>(im, x0, y0 - r, CWn, block_interior(y0 - r), fvs);
  __syncthreads();   // the previous group's readers are done with both buffers
  for (int qq = 0; qq < QB; qq += DV) {
#pragma unroll
    for (int u = 0; u < DV; ++u) {
      const int q = qq + u;
      if (q < QB) {
        float* buf = sbuf + (q & 1) * (kF32Ch * 16 * PC);
        const int row0 = y0 - r + 16 * q;
        const int pb = q - (DV - 1);
        float fo[4], nv[4], dv[4];
        if (pb >= 0) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            nv[v] = Ns[pb * 256 + 64 * v + lane];
            if (HK) dv[v] = Ds[pb * 256 + 64 * v + lane];
          }
          chk_nd(im, Ns + pb * 256 + lane, 193);
          chk_nd(im, Ds + pb * 256 + lane, 193);
        }
        if (HK) {
          if (rows_in) {
            const float* const p = fo_base + static_cast<size_t>(16 * max(pb, 0)) * ld;
            chk_img(im, y0 + 16 * max(pb, 0) + 4 * lk + 3, gxo);
#pragma unroll
            for (int v = 0; v < 4; ++v) fo[v] = p[v * ld];
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int gy = min(max(y0 + 16 * pb + 4 * lk + v, 0), im.H - 1);
              chk_img(im, gy, gxo);
              fo[v] = im.in[gy * ld + gxo];
            }
          }
        }
        if (block_interior(row0))
          f32s_stage<G, IW, true>(im, kinv, x0, row0, CWn, PC, buf, fvs);
        else
          f32s_stage<G, IW, false>(im, kinv, x0, row0, CWn, PC, buf, fvs);
        const int rown = y0 - r + 16 * ((q + 1 < QB) ? q + 1 : q);
        stage_fetch<IW>(im, x0, rown, CWn, block_interior(rown), fvs);
        __syncthreads();
        // ---- horizontal pass of this wave's strip, from LDS ----
        const float* arow = buf + hrow_of_lane(li) * PC + 16 * wave + SH * lk;
        // Pinned row pointers halve the kernel's vector adds; measured at
        // 4096^2 they gain 0.8-1.9% where SH is not a multiple of 4 (theta
        // = 6, 7, 10, 12) and lose 0.5-0.8% where it is (theta = 8, 5).
        constexpr bool PIN = SH % 4 != 0;
        const float* ag[G];
#pragma unroll
        for (int g = 0; g < G; ++g)
          ag[g] = PIN ? lds_pinned(arow + g * 16 * PC) : arow + g * 16 * PC;
        chk_lds(im, ag[0], 4);
        chk_lds(im, ag[G - 1] + SH - 1, 4);
        f4 acc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < SH; ++s) {
          const float bh = TREG ? btr[s] : Bt[s * 64 + lane];
#pragma unroll
          for (int g = 0; g < G; ++g)
            acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(ag[g][s], bh, acc[g], 0, 0, 0);
        }
#pragma unroll
        for (int g = 0; g < G; ++g) ring[u][g] = acc[g];
        tags.set(u, q);
        // ---- vertical pass, output block pb ----
        if (pb >= 0) {
          f4 vacc[G];
#pragma unroll
          for (int g = 0; g < G; ++g) vacc[g] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int d = 0; d < DV; ++d) {
            const int slot = (u + 1 + d) % DV;
            tags.check(im, slot, pb + d);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              if (4 * d + v >= SH) break;   // all-zero slices
              const float av = TREG ? atr[d * 4 + v] : At[(d * 4 + v) * 64 + lane];
#pragma unroll
              for (int g = 0; g < G; ++g)
                vacc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, ring[slot][g][v], vacc[g],
                                                               0, 0, 0);
            }
          }
          // f's term first, then frequency k's: the additions of two
          // separate passes
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if (HF) nv[v] = fmaf(c0, vacc[0][v], nv[v]);
            if (HK) {
              float sn, cs;
              sincos_rev(kinv * fo[v], &sn, &cs);
              nv[v] = fmaf(ck, fmaf(cs, vacc[g0][v], sn * vacc[g0 + 1][v]), nv[v]);
              dv[v] = fmaf(ck, fmaf(cs, vacc[g0 + 2][v], sn * vacc[g0 + 3][v]), dv[v]);
            }
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            Ns[pb * 256 + 64 * v + lane] = nv[v];
            if (HK) Ds[pb * 256 + 64 * v + lane] = dv[v];
          }
        }
      }
    }
  }
}

// nd: this workgroup's share of the workspace, 2 nblk 256 floats per wave.
template <int SH, int NW>
__device__ __forceinline__ void f32s_tile(const Img& im, int tx, int ty, int nblk,
                                          const float* tbl, const float* Bt, const float* At,
                                          float* sbuf, int PC, float* nd) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  float* Ns = nd + wave * 2 * nblk * 256;
  float* Ds = Ns + nblk * 256;
  const int x0 = tx * (NW * MSTRIP);
  const int y0 = ty * 16 * nblk;
  // zero both staging buffers: columns past the items are read by steps
  // whose taps are zero, so they must hold finite values
  {
    float4* z = reinterpret_cast<float4*>(sbuf);
    const int n16 = 2 * kF32Ch * 16 * PC / 4;
    for (int i = threadIdx.x; i < n16; i += 64 * NW) {
      chk_lds(im, z + i, 16);
      z[i] = float4{0.f, 0.f, 0.f, 0.f};
    }
  }
  init_nd(im, tbl, x0 + wave * MSTRIP, y0, nblk, Ns, Ds, lane);
  constexpr int DV = (SH + 3) / 4;
  constexpr bool TREG = DV <= 5;
  float btr[SH], atr[4 * DV];
  if (TREG) {
#pragma unroll
    for (int s = 0; s < SH; ++s) btr[s] = Bt[s * 64 + lane];
#pragma unroll
    for (int i = 0; i < 4 * DV; ++i) atr[i] = At[i * 64 + lane];
  }
  if (im.K == 1) {
    f32s_group<SH, NW, 1, TREG>(im, 0, x0, y0, nblk, tbl, Bt, At, sbuf, PC, Ns, Ds, btr, atr);
  } else {
    f32s_group<SH, NW, 5, TREG>(im, 1, x0, y0, nblk, tbl, Bt, At, sbuf, PC, Ns, Ds, btr, atr);
    for (int k = 2; k < im.K; ++k)
      f32s_group<SH, NW, 4, TREG>(im, k, x0, y0, nblk, tbl, Bt, At, sbuf, PC, Ns, Ds, btr, atr);
  }
  store_nd(im, x0 + wave * MSTRIP, y0, nblk, Ns, Ds, lane);
}

// GND = false: N and D of the tile live in LDS (the single-image and batch
// kernels).  GND = true: they live in a global workspace, which frees the
// LDS for much taller tiles (fewer halo blocks per output block); the
// block's N and D are then fetched at the head of the block, a whole block
// of matrix work ahead of the fold, and the vertical pass uses the K = 16
// product (one horizontal block per operand: no register moves to pair
// blocks, fewer registers).
template <typename OT, int DV, int G, int NW, bool GND = false>
__device__ __forceinline__ void staged_group(const Img& im, int k, float shift, int x0, int y0,
                                             int nblk, const float* tbl,
                                             typename Stage<OT>::T* sbuf, float* Ns,
                                             float* Ds) {
  using S = Stage<OT>;
  typedef typename S::v8 v8;
  typedef typename S::T o4 __attribute__((ext_vector_type(4)));
  constexpr bool HF = group_has_f<G>();      // channel f leads the group
  constexpr int NF = group_freqs<G>();       // frequencies k .. k+NF-1
  constexpr int SCH = staged_channels<OT, DV, GND>();
  static_assert(G == (HF ? 1 : 0) + 4 * NF && G <= SCH, "bad channel group");
  // sub-groups: {f} when present, then one per frequency (4 channels)
  constexpr int NSG = (HF ? 1 : 0) + NF;
  // the merged groups run sub-group by sub-group (fewer accumulators live
  // at once); one-frequency groups keep their all-channels-at-once order
  constexpr bool SUB = staged_merge<OT, GND>() || G == 5;
  auto sg_first = [](int sg) { return HF ? (sg == 0 ? 0 : 4 * sg - 3) : 4 * sg; };
  auto sg_size = [](int sg) { return (HF && sg == 0) ? 1 : 4; };
  constexpr int SHS = (DV + 1) / 2;          // 32-column horizontal steps
  constexpr int NV = (DV + 1) / 2;           // vertical MFMAs (2 blocks each)
  constexpr int PC = stage_pitch(stage_width<DV, NW>());
  const float* gS = tbl;
  const float* cS = tbl + 64;
  const int r = im.r;
  const int CWn = 16 * NW + 2 * r;           // columns meeting non-zero taps
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  float kinv[NF > 0 ? NF : 1], ck[NF > 0 ? NF : 1];
#pragma unroll
  for (int q = 0; q < NF; ++q) {
    kinv[q] = static_cast<float>(k + q) * im.inv_period;
    ck[q] = cS[k + q];
  }
  const float c0 = cS[0];
  const int x0w = x0 + wave * MSTRIP;
  const int QB = nblk + DV - 1;
  constexpr int IW = stage_item_width<DV, NW>();
  static_assert(16 * NW + 16 * (DV - 1) + IW - 1 <= PC, "staged items overrun the pitch");
  const bool cols_in = x0 - r >= 0 && x0 - r + IW * ((CWn + IW - 1) / IW) <= im.W;

  // horizontal weights: lane (lk, n = li), element j <-> column 32s + 8lk + j
  constexpr int NS = S::kParts;              // words per staged value
  v8 Bw[SHS][NS];
#pragma unroll
  for (int s = 0; s < SHS; ++s)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float w = tap(gS, 32 * s + 8 * lk + j - r - li, r);
      Bw[s][0][j] = S::cvt(w);
      if (NS == 2) Bw[s][NS - 1][j] = S::cvt(w - static_cast<float>(Bw[s][0][j]));
    }
  // (two-word workspace forms with f merged: built by wave 0 into the LDS
  // after the vertical slices and read back per horizontal step; every
  // group writes the same values)
  constexpr bool kHtapLds = staged_fmerge2<OT, DV, GND>();
  v8* const htap = reinterpret_cast<v8*>(reinterpret_cast<char*>(sbuf) +
                                         staged_stage_bytes<OT, DV, NW, GND>() +
                                         staged_vtap_bytes<OT, DV, NW>());
  if (kHtapLds && wave == 0)
#pragma unroll
    for (int s = 0; s < SHS; ++s)
#pragma unroll
      for (int h = 0; h < NS; ++h) {
        chk_lds(im, htap + (s * NS + h) * 64 + lane, sizeof(v8));
        htap[(s * NS + h) * 64 + lane] = Bw[s][h];
      }
  // vertical weights: MFMA t pairs H blocks 2t (elements 0..3) and 2t+1
  // (elements 4..7); element j <-> H row 16 (2t + j/4) + 4 lk + j%4
  // (two-word modes: built by wave 0 into the LDS table after the staging
  // buffers and read back per vertical step)
  // (K = 16 form, GND: one operand per H block d, element j <-> H row
  // 16 d + 4 lk + j; the table fits in the same LDS bytes)
  constexpr bool kVtapLds = staged_vtap_in_lds<OT, NW>();
  static_assert(!GND || !kVtapLds ||
                    DV * NS * 64 * sizeof(o4) <= staged_vtap_bytes<OT, DV, NW>(),
                "the K = 16 tap table must fit the vertical tap area");
  v8 Aw[GND ? 1 : NV][NS];
  o4 Aw4[GND ? DV : 1][NS];
  v8* const vtap = reinterpret_cast<v8*>(reinterpret_cast<char*>(sbuf) +
                                         staged_stage_bytes<OT, DV, NW, GND>());
  o4* const vtap4 = reinterpret_cast<o4*>(vtap);
  if (!kVtapLds || wave == 0) {
    if constexpr (GND) {
#pragma unroll
      for (int d = 0; d < DV; ++d)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float w = tap(gS, 16 * d + 4 * lk + j - r - li, r);
          Aw4[d][0][j] = S::cvt(w);
          if (NS == 2) Aw4[d][NS - 1][j] = S::cvt(w - static_cast<float>(Aw4[d][0][j]));
        }
      if (kVtapLds)
#pragma unroll
        for (int d = 0; d < DV; ++d)
#pragma unroll
          for (int h = 0; h < NS; ++h) {
            chk_lds(im, vtap4 + (d * NS + h) * 64 + lane, sizeof(o4));
            vtap4[(d * NS + h) * 64 + lane] = Aw4[d][h];
          }
    } else {
#pragma unroll
      for (int t = 0; t < NV; ++t)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int blk = 2 * t + (j >> 2);
          const float w = blk < DV ? tap(gS, 16 * blk + 4 * lk + (j & 3) - r - li, r) : 0.f;
          Aw[t][0][j] = S::cvt(w);
          if (NS == 2) Aw[t][NS - 1][j] = S::cvt(w - static_cast<float>(Aw[t][0][j]));
        }
      if (kVtapLds)
#pragma unroll
        for (int t = 0; t < NV; ++t)
#pragma unroll
          for (int h = 0; h < NS; ++h) {
            chk_lds(im, vtap + (t * NS + h) * 64 + lane, sizeof(v8));
            vtap[(t * NS + h) * 64 + lane] = Aw[t][h];
          }
    }
  }

  o4 ring[DV][NS][G];
  RingTags<DV> tags;
  // check builds: the horizontal reads of step s (columns 16 wave + 32 s +
  // 8 lk + 0..7 of buffer row li) stay in the row and in the LDS, and the
  // taps they meet join them to output columns inside their windows
  FOBF_CHK(im, 16 * wave + 32 * (SHS - 1) + 8 * lk + 8 <= PC, FOBF_CHECK_HALO_H);
#if FOBF_CHECKS
#pragma unroll
  for (int s = 0; s < SHS; ++s)
#pragma unroll
    for (int j = 0; j < 8; ++j)
      chk_htap(im, static_cast<float>(Bw[s][0][j]), 32 * s + 8 * lk + j, li);
#endif
  auto chk_hread = [&](const typename S::T* rowp, int s) {
    if (s == 0 || s == SHS - 1) chk_lds(im, rowp, 8 * sizeof(typename S::T));
  };
  // check builds: the vertical taps met by ring block d (K = 16 operand:
  // element j <-> H row 16 d + 4 lk + j; K = 32 operand t: element j <->
  // H row 16 (2t + j/4) + 4 lk + j%4), and the blocks the slots hold
  // (the taps once per group, as every block reads them; the slots per
  // block)
#if FOBF_CHECKS
  if (!kVtapLds || wave == 0) {
    if constexpr (GND) {
#pragma unroll
      for (int d = 0; d < DV; ++d)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          chk_vtap(im, static_cast<float>(Aw4[d][0][j]), 16 * d + 4 * lk + j, li);
    } else {
#pragma unroll
      for (int t = 0; t < NV; ++t)
#pragma unroll
        for (int j = 0; j < 8; ++j)
          chk_vtap(im, static_cast<float>(Aw[t][0][j]),
                   16 * (2 * t + (j >> 2)) + 4 * lk + (j & 3), li);
    }
  }
#endif
  auto chk_vread4 = [&](const o4&, int d, int slot, int pb) { tags.check(im, slot, pb + d); };
  auto chk_vread8 = [&](const v8&, int t, int slot0, int slot1, int pb) {
    tags.check(im, slot0, pb + 2 * t);
    if (2 * t + 1 < DV) tags.check(im, slot1, pb + 2 * t + 1);
  };
  auto block_interior = [&](int row0) { return cols_in && row0 >= 0 && row0 + 16 <= im.H; };
  // the fold's pixel values: where every output row of the tile lies in
  // the image, block pb's four rows are at a fixed stride from one base
  // (blocks with pb < 0 fold nothing: they read block 0's)
  const size_t ldi = static_cast<size_t>(im.ld_in);
  const bool rows_in = y0 + 16 * nblk <= im.H;
  const float* const fo_base =
      im.in + static_cast<size_t>(min(y0 + 4 * lk, im.H - 1)) * ldi + min(x0w + li, im.W - 1);
  float fvs[IW];
  stage_fetch<IW>(im, x0, y0 - r, CWn, block_interior(y0 - r), fvs);
  __syncthreads();   // the previous group's readers are done with both buffers
  for (int qq = 0; qq < QB; qq += DV) {
#pragma unroll
    for (int u = 0; u < DV; ++u) {
      const int q = qq + u;
      if (q < QB) {
        constexpr int NBUF = staged_bufs<OT, NW, GND>();
        typename S::T* buf = sbuf + (NBUF == 2 ? (q & 1) : 0) * (NS * SCH * 16 * PC);
        const int row0 = y0 - r + 16 * q;
        const int pb = q - (DV - 1);
        // output-pixel values for this block's fold, loaded before the
        // staging so that they arrive during the block's matrix work (rows
        // clamped: blocks with pb < 0 fold nothing)
        float fo[4];
        float nv[4], dv[4];
        if (GND && pb >= 0) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            nv[v] = Ns[pb * 256 + 64 * v + lane];
            if (NF > 0) dv[v] = Ds[pb * 256 + 64 * v + lane];
          }
          chk_nd(im, Ns + pb * 256 + lane, 193);
          chk_nd(im, Ds + pb * 256 + lane, 193);
        }
        if (NF > 0) {
          if (rows_in) {
            const float* const p = fo_base + static_cast<size_t>(16 * max(pb, 0)) * ldi;
            chk_img(im, y0 + 16 * max(pb, 0) + 4 * lk + 3, min(x0w + li, im.W - 1));
#pragma unroll
            for (int v = 0; v < 4; ++v) fo[v] = p[v * ldi];
          } else {
            const int gx = min(x0w + li, im.W - 1);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int gy = min(max(y0 + 16 * pb + 4 * lk + v, 0), im.H - 1);
              chk_img(im, gy, gx);
              fo[v] = im.in[static_cast<size_t>(gy) * ldi + gx];
            }
          }
        }
        if (block_interior(row0))
          stage_block<OT, G, IW, true, SCH>(im, k, shift, x0, row0, CWn, PC, buf, fvs);
        else
          stage_block<OT, G, IW, false, SCH>(im, k, shift, x0, row0, CWn, PC, buf, fvs);
        // next block's loads (the last block reloads its own: branch-free)
        const int rown = y0 - r + 16 * ((q + 1 < QB) ? q + 1 : q);
        stage_fetch<IW>(im, x0, rown, CWn, block_interior(rown), fvs);
        __syncthreads();
        if constexpr (!SUB) {
        // ---- horizontal pass of this wave's strip ----
        f4 acc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < SHS; ++s)
#pragma unroll
          for (int g = 0; g < G; ++g) {
            v8 a[NS];
            if (g == 0) chk_hread(buf + li * PC + 16 * wave + 32 * s + 8 * lk, s);
#pragma unroll
            for (int h = 0; h < NS; ++h)
              a[h] = *reinterpret_cast<const v8*>(buf + ((h * SCH + g) * 16 + li) * PC +
                                                  16 * wave + 32 * s + 8 * lk);
            // hi*hi (+ lo*hi + hi*lo when values are split)
#pragma unroll
            for (int ha = 0; ha < NS; ++ha)
#pragma unroll
              for (int hb = 0; hb + ha < NS; ++hb)
                acc[g] = S::mfma(a[ha], kHtapLds ? htap[(s * NS + hb) * 64 + lane] : Bw[s][hb],
                                 acc[g]);
          }
        // one buffer: every wave is done reading it before the next block
        // is staged into it
        if (NBUF == 1) __syncthreads();
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            ring[u][0][g][v] = S::cvt(acc[g][v]);
            if (NS == 2)
              ring[u][NS - 1][g][v] = S::cvt(acc[g][v] - static_cast<float>(ring[u][0][g][v]));
          }
        tags.set(u, q);

        // ---- vertical pass, output block pb = q - DV + 1 ----
        if (pb >= 0) {
          f4 vacc[G];
#pragma unroll
          for (int g = 0; g < G; ++g) vacc[g] = f4{0.f, 0.f, 0.f, 0.f};
          if constexpr (GND) {
#pragma unroll
            for (int d = 0; d < DV; ++d) {
              const int slot = (u + 1 + d) % DV;
              o4 aw[NS];
#pragma unroll
              for (int h = 0; h < NS; ++h)
                aw[h] = kVtapLds ? vtap4[(d * NS + h) * 64 + lane] : Aw4[d][h];
              chk_vread4(aw[0], d, slot, pb);
#pragma unroll
              for (int g = 0; g < G; ++g)
#pragma unroll
                for (int ha = 0; ha < NS; ++ha)
#pragma unroll
                  for (int hb = 0; hb + ha < NS; ++hb)
                    vacc[g] = S::mfma16(aw[ha], ring[slot][hb][g], vacc[g]);
            }
          } else {
#pragma unroll
          for (int t = 0; t < NV; ++t) {
            const int b0 = 2 * t, b1 = (2 * t + 1 < DV) ? 2 * t + 1 : 2 * t;
            v8 aw[NS];
#pragma unroll
            for (int h = 0; h < NS; ++h) aw[h] = kVtapLds ? vtap[(t * NS + h) * 64 + lane] : Aw[t][h];
            chk_vread8(aw[0], t, (u + 1 + b0) % DV, (u + 1 + b1) % DV, pb);
#pragma unroll
            for (int g = 0; g < G; ++g) {
              v8 b[NS];
#pragma unroll
              for (int h = 0; h < NS; ++h) {
                const o4 e0 = ring[(u + 1 + b0) % DV][h][g];
                const o4 e1 = ring[(u + 1 + b1) % DV][h][g];
                b[h] = v8{e0[0], e0[1], e0[2], e0[3], e1[0], e1[1], e1[2], e1[3]};
              }
#pragma unroll
              for (int ha = 0; ha < NS; ++ha)
#pragma unroll
                for (int hb = 0; hb + ha < NS; ++hb) vacc[g] = S::mfma(aw[ha], b[hb], vacc[g]);
            }
          }
          }
          // fold (all reads of N, D before the writes they may alias)
          float* const nrow = Ns + pb * 256 + lane;
          float* const drow = Ds + pb * 256 + lane;
          if (!GND) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              nv[v] = nrow[64 * v];
              if (NF > 0) dv[v] = drow[64 * v];
            }
            chk_nd(im, nrow, 193);
            chk_nd(im, drow, 193);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if (HF) {
              nv[v] = fmaf(c0, vacc[0][v], nv[v]);
            } else {
              float sn, cs;
              sincos_rev(kinv[0] * fo[v], &sn, &cs);
              nv[v] = fmaf(ck[0], fmaf(cs, vacc[0][v], sn * vacc[1][v]), nv[v]);
              dv[v] = fmaf(ck[0], fmaf(cs, vacc[2][v], sn * vacc[3][v]), dv[v]);
            }
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            nrow[64 * v] = nv[v];
            if (NF > 0) drow[64 * v] = dv[v];
          }
        }
        } else {
        // ---- horizontal pass of this wave's strip, one sub-group (f, or
        // one frequency's four channels) at a time, each converted into the
        // ring right away (fewer accumulators live at once) ----
#pragma unroll
        for (int sg = 0; sg < NSG; ++sg) {
          const int gb = sg_first(sg), gn = sg_size(sg);
          f4 acc[4];
#pragma unroll
          for (int i = 0; i < gn; ++i) acc[i] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int s = 0; s < SHS; ++s)
#pragma unroll
            for (int i = 0; i < gn; ++i) {
              v8 a[NS];
              if (sg == 0 && i == 0) chk_hread(buf + li * PC + 16 * wave + 32 * s + 8 * lk, s);
#pragma unroll
              for (int h = 0; h < NS; ++h)
                a[h] = *reinterpret_cast<const v8*>(buf + ((h * SCH + gb + i) * 16 + li) * PC +
                                                    16 * wave + 32 * s + 8 * lk);
              // hi*hi (+ lo*hi + hi*lo when values are split)
#pragma unroll
              for (int ha = 0; ha < NS; ++ha)
#pragma unroll
                for (int hb = 0; hb + ha < NS; ++hb)
                  acc[i] = S::mfma(a[ha], kHtapLds ? htap[(s * NS + hb) * 64 + lane] : Bw[s][hb],
                                   acc[i]);
            }
#pragma unroll
          for (int i = 0; i < gn; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              ring[u][0][gb + i][v] = S::cvt(acc[i][v]);
              if (NS == 2)
                ring[u][NS - 1][gb + i][v] =
                    S::cvt(acc[i][v] - static_cast<float>(ring[u][0][gb + i][v]));
            }
        }
        tags.set(u, q);
        // one buffer: every wave is done reading it before the next block
        // is staged into it
        if (NBUF == 1) __syncthreads();

        // ---- vertical pass, output block pb = q - DV + 1, and the fold,
        // sub-group by sub-group ----
        if (pb >= 0) {
          // fold (all reads of N, D before the writes they may alias)
          float* const nrow = Ns + pb * 256 + lane;
          float* const drow = Ds + pb * 256 + lane;
          if (!GND) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              nv[v] = nrow[64 * v];
              if (NF > 0) dv[v] = drow[64 * v];
            }
            chk_nd(im, nrow, 193);
            chk_nd(im, drow, 193);
          }
#pragma unroll
          for (int sg = 0; sg < NSG; ++sg) {
            const int gb = sg_first(sg), gn = sg_size(sg);
            f4 vacc[4];
#pragma unroll
            for (int i = 0; i < gn; ++i) vacc[i] = f4{0.f, 0.f, 0.f, 0.f};
            if constexpr (GND) {
#pragma unroll
              for (int d = 0; d < DV; ++d) {
                const int slot = (u + 1 + d) % DV;
                o4 aw[NS];
#pragma unroll
                for (int h = 0; h < NS; ++h)
                  aw[h] = kVtapLds ? vtap4[(d * NS + h) * 64 + lane] : Aw4[d][h];
                if (sg == 0) chk_vread4(aw[0], d, slot, pb);
#pragma unroll
                for (int i = 0; i < gn; ++i)
#pragma unroll
                  for (int ha = 0; ha < NS; ++ha)
#pragma unroll
                    for (int hb = 0; hb + ha < NS; ++hb)
                      vacc[i] = S::mfma16(aw[ha], ring[slot][hb][gb + i], vacc[i]);
              }
            } else {
#pragma unroll
              for (int t = 0; t < NV; ++t) {
                const int b0 = 2 * t, b1 = (2 * t + 1 < DV) ? 2 * t + 1 : 2 * t;
                v8 aw[NS];
#pragma unroll
                for (int h = 0; h < NS; ++h)
                  aw[h] = kVtapLds ? vtap[(t * NS + h) * 64 + lane] : Aw[t][h];
                if (sg == 0) chk_vread8(aw[0], t, (u + 1 + b0) % DV, (u + 1 + b1) % DV, pb);
#pragma unroll
                for (int i = 0; i < gn; ++i) {
                  v8 b[NS];
#pragma unroll
                  for (int h = 0; h < NS; ++h) {
                    const o4 e0 = ring[(u + 1 + b0) % DV][h][gb + i];
                    const o4 e1 = ring[(u + 1 + b1) % DV][h][gb + i];
                    b[h] = v8{e0[0], e0[1], e0[2], e0[3], e1[0], e1[1], e1[2], e1[3]};
                  }
#pragma unroll
                  for (int ha = 0; ha < NS; ++ha)
#pragma unroll
                    for (int hb = 0; hb + ha < NS; ++hb)
                      vacc[i] = S::mfma(aw[ha], b[hb], vacc[i]);
                }
              }
            }
            // f first, then the frequencies in order: the additions into
            // N and D are those of one group per frequency
            if (HF && sg == 0) {
#pragma unroll
              for (int v = 0; v < 4; ++v) nv[v] = fmaf(c0, vacc[0][v], nv[v]);
            } else {
              const int qf = max(0, HF ? sg - 1 : sg);
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                float sn, cs;
                sincos_rev(kinv[qf] * fo[v], &sn, &cs);
                nv[v] = fmaf(ck[qf], fmaf(cs, vacc[0][v], sn * vacc[1][v]), nv[v]);
                dv[v] = fmaf(ck[qf], fmaf(cs, vacc[2][v], sn * vacc[3][v]), dv[v]);
              }
            }
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            nrow[64 * v] = nv[v];
            if (NF > 0) drow[64 * v] = dv[v];
          }
        }
        }
      }
    }
  }
}

// nd: N and D of the tile's waves, 2 * nblk * 256 floats per wave (in LDS,
// or for GND this workgroup's share of the global workspace).
template <typename OT, int DV, int NW, bool GND = false>
__device__ __forceinline__ void staged_tile(const Img& im, int tx, int ty, int nblk,
                                            const float* tbl, typename Stage<OT>::T* sbuf,
                                            float* nd) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int TYo = 16 * nblk;
  float* Ns = nd + wave * 2 * nblk * 256;
  float* Ds = Ns + nblk * 256;
  const int x0 = tx * (NW * MSTRIP);
  const int y0 = ty * TYo;
  const int x0w = x0 + wave * MSTRIP;
  // zero both staging buffers: the columns past 16 NW + 2r are multiplied
  // by zero taps and are never written, so they must hold finite values
  {
    float4* z = reinterpret_cast<float4*>(sbuf);
    const int n16 = static_cast<int>(staged_stage_bytes<OT, DV, NW, GND>() / 16);
    for (int i = threadIdx.x; i < n16; i += 64 * NW) {
      chk_lds(im, z + i, 16);
      z[i] = float4{0.f, 0.f, 0.f, 0.f};
    }
  }
  // Staged channels carry (f - m) instead of f, m = f at the tile centre:
  // the numerator becomes N - m D exactly, so out = N'/D + m, and the
  // magnitudes rounded to the staging type shrink to the local contrast.
  chk_img(im, min(y0 + TYo / 2, im.H - 1), min(x0 + NW * MSTRIP / 2, im.W - 1));
  const float shift = im.in[static_cast<size_t>(min(y0 + TYo / 2, im.H - 1)) * im.ld_in +
                            min(x0 + NW * MSTRIP / 2, im.W - 1)];
  init_nd(im, tbl, x0w, y0, nblk, Ns, Ds, lane);
  if constexpr (staged_merge<OT, GND>()) {
    // {f, 1}, {2, 3}, {4, 5}, .. (and a last single frequency for even K)
    if (im.K == 1) {
      staged_group<OT, DV, 1, NW, GND>(im, 0, shift, x0, y0, nblk, tbl, sbuf, Ns, Ds);
    } else {
      staged_group<OT, DV, 5, NW, GND>(im, 1, shift, x0, y0, nblk, tbl, sbuf, Ns, Ds);
      int k = 2;
      for (; k + 1 < im.K; k += 2)
        staged_group<OT, DV, 8, NW, GND>(im, k, shift, x0, y0, nblk, tbl, sbuf, Ns, Ds);
      if (k < im.K)
        staged_group<OT, DV, 4, NW, GND>(im, k, shift, x0, y0, nblk, tbl, sbuf, Ns, Ds);
    }
  } else if constexpr (staged_fmerge2<OT, DV, GND>()) {
    // {f, 1}, 2, 3, ..
    if (im.K == 1) {
      staged_group<OT, DV, 1, NW, GND>(im, 0, shift, x0, y0, nblk, tbl, sbuf, Ns, Ds);
    } else {
      staged_group<OT, DV, 5, NW, GND>(im, 1, shift, x0, y0, nblk, tbl, sbuf, Ns, Ds);
      for (int k = 2; k < im.K; ++k)
        staged_group<OT, DV, 4, NW, GND>(im, k, shift, x0, y0, nblk, tbl, sbuf, Ns, Ds);
    }
  } else {
    staged_group<OT, DV, 1, NW, GND>(im, 0, shift, x0, y0, nblk, tbl, sbuf, Ns, Ds);
    for (int k = 1; k < im.K; ++k)
      staged_group<OT, DV, 4, NW, GND>(im, k, shift, x0, y0, nblk, tbl, sbuf, Ns, Ds);
  }
  store_nd(im, x0w, y0, nblk, Ns, Ds, lane, shift);
}

// =========================================================================
// launch helpers shared by the single-image launch files
// =========================================================================

// Workgroup width of the staged kernels: eight strips (wider tiles share
// more of the horizontal halo's channel work), except for the two-word
// bf16 staging at the largest radii (DV = 7), whose registers spill at
// eight waves: there four are faster (4096^2, theta = 15: 2.23 vs 3.07 ms;
// at theta = 10 and 13 eight win, 1.28 vs 1.70 and 1.81 vs 1.92 ms).
template <typename OT, int DV>
constexpr int staged_waves() { return (Stage<OT>::kParts == 2 && DV >= 7) ? 4 : 8; }

constexpr int kWsWaves = 8;   // strips per workgroup of the workspace forms

template <typename KernelT>
inline void allow_big_lds(KernelT kernel) {
  hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

// 1-D grid: tiles (nw strips wide) rounded up to a multiple of the 8 XCDs
inline unsigned padded_blocks(const ImageParams& p, int nblk, int nw = MWAVES) {
  const long ntx = (p.W + nw * MSTRIP - 1) / (nw * MSTRIP);
  const long nty = (p.H + 16 * nblk - 1) / (16 * nblk);
  return static_cast<unsigned>(((ntx * nty + 7) / 8) * 8);
}

// Compute units of the current device, looked up once per device.
inline int device_cus() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int n = cache[dev].load(std::memory_order_relaxed);
  if (n == 0) {
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
      n = 256;
    cache[dev].store(n, std::memory_order_relaxed);
  }
  return n;
}

// Tile height (at most the tuned nblk) for an image with only a few tiles
// per workgroup slot (per_cu resident workgroups of nw strips per CU):
// there the tiles run in a few rounds of one per slot, each round as long
// as one tile's chain of nblk + DV - 1 blocks, so the height that
// minimises rounds x chain wins even though shorter tiles recompute more
// halo rows (128^2 .. 1024^2 images: 2-3x faster).  Images with many
// rounds keep the tuned height.
inline int fill_nblk(int H, int W, int nblk, int nw, int per_cu, int dv) {
  const long ntx = (W + nw * MSTRIP - 1) / (nw * MSTRIP);
  const long slots = static_cast<long>(device_cus()) * per_cu;
  auto tiles = [&](int n) { return ntx * ((H + 16L * n - 1) / (16L * n)); };
  if (tiles(nblk) >= 4 * slots) return nblk;
  int best = nblk;
  long best_cost = ((tiles(nblk) + slots - 1) / slots) * (nblk + dv - 1);
  for (int n = nblk - 1; n >= 1; --n) {
    const long cost = ((tiles(n) + slots - 1) / slots) * (n + dv - 1);
    if (cost < best_cost) best = n, best_cost = cost;
  }
  return best;
}

inline fobf_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(FOBF_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return FOBF_OK;
}

}  // namespace
}  // namespace fobf
