// Workspace forms of the single-image kernels (fobf_filter_ws): each
// tile's running N and D live in a caller-provided device workspace instead
// of the LDS, which frees the LDS for 512-row tiles (far fewer vertical halo
// blocks) and, for float32, for channels staged once per workgroup.  The
// device building blocks are in fobf_tiles.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <utility>

#include "fobf_tiles.h"

namespace fobf {
namespace {

// Tall-tile form of the staged kernel: each tile's N and D live in a global
// workspace (2 nblk 256 floats per wave, tiles in row-major order), so the
// LDS holds only the staging buffer and the tile can be 512 rows tall.
template <typename OT, int DV>
__global__ __launch_bounds__((64 * staged_waves<OT, DV>())) void mfma_staged_ws_kernel(
    ImageParams p, int nblk, float* work) {
  constexpr int NW = staged_waves<OT, DV>();
  extern __shared__ float lds[];
  const int ntx = (p.W + NW * MSTRIP - 1) / (NW * MSTRIP);
  const int nty = (p.H + 16 * nblk - 1) / (16 * nblk);
  int tx, ty;
  if (!tile_of_block(blockIdx.x, gridDim.x, ntx, nty, &tx, &ty)) return;
  float* tbl = lds;
  typename Stage<OT>::T* sbuf = reinterpret_cast<typename Stage<OT>::T*>(lds + LDS_TABLE);
  float* nd = work + (static_cast<size_t>(ty) * ntx + tx) * (NW * 2 * 256) * nblk;
  const Img im = FOBF_IMG(p);
  poison_lds(im);
  FOBF_LOAD_TABLES(p, tbl);
  __syncthreads();
  staged_tile<OT, DV, NW, true>(im, tx, ty, nblk, tbl, sbuf, nd);
}

// float32 workspace form: channels staged per workgroup, 512-row tiles.
template <int SH>
__global__ __launch_bounds__(64 * kWsWaves) void mfma_f32_ws_kernel(ImageParams p, int nblk,
                                                                   float* work) {
  constexpr int DV = (SH + 3) / 4;
  constexpr int NW = kWsWaves;
  extern __shared__ float lds[];
  const int ntx = (p.W + NW * MSTRIP - 1) / (NW * MSTRIP);
  const int nty = (p.H + 16 * nblk - 1) / (16 * nblk);
  int tx, ty;
  if (!tile_of_block(blockIdx.x, gridDim.x, ntx, nty, &tx, &ty)) return;
  float* tbl = lds;
  float* Bt = lds + LDS_TABLE;
  float* At = Bt + 4 * DV * 64;
  float* sbuf = At + 4 * DV * 64;
  const int PC = f32s_pitch(SH, NW, p.r, stage_item_width<DV, NW>());
  float* nd = work + (static_cast<size_t>(ty) * ntx + tx) * (NW * 2 * 256) * nblk;
  const Img im = FOBF_IMG(p);
  poison_lds(im);
  FOBF_LOAD_TABLES(p, tbl);
  __syncthreads();
  build_f32_tables<SH>(im, tbl, p.r, Bt, At);
  __syncthreads();
  f32s_tile<SH, NW>(im, tx, ty, nblk, tbl, Bt, At, sbuf, PC, nd);
}

template <typename OT, int DV>
fobf_status launch_staged_ws_dv(const ImageParams& p, int nblk, float* work, void* stream) {
  static const bool once = (allow_big_lds(mfma_staged_ws_kernel<OT, DV>), true);
  (void)once;
  constexpr int NW = staged_waves<OT, DV>();
  static_assert(NW == kWsWaves, "the workspace form runs eight strips");
  constexpr size_t lds = sizeof(float) * LDS_TABLE + staged_buf_bytes<OT, DV, NW, true>();
  static_assert(lds <= 160 * 1024, "staging buffers exceed the LDS");
  dim3 grid(padded_blocks(p, nblk, NW));
  ImageParams q = p;
  q.lds_bytes = static_cast<int>(lds);
  hipLaunchKernelGGL((mfma_staged_ws_kernel<OT, DV>), grid, dim3(64 * NW), lds,
                     static_cast<hipStream_t>(stream), q, nblk, work);
  return check_launch("mfma_staged_ws_kernel");
}

template <int SH>
fobf_status launch_f32_ws_sh(const ImageParams& p, int nblk, float* work, void* stream) {
  constexpr int DV = (SH + 3) / 4;
  static const bool once = (allow_big_lds(mfma_f32_ws_kernel<SH>), true);
  (void)once;
  const int PC = f32s_pitch(SH, kWsWaves, p.r, stage_item_width<DV, kWsWaves>());
  const size_t lds = sizeof(float) * (LDS_TABLE + 8 * DV * 64 +
                                      2 * static_cast<size_t>(kF32Ch) * 16 * PC);
  if (lds > 160 * 1024) return fail(FOBF_EINTERNAL, "fobf_filter_ws: staging exceeds the LDS");
  dim3 grid(padded_blocks(p, nblk, kWsWaves));
  ImageParams q = p;
  q.lds_bytes = static_cast<int>(lds);
  hipLaunchKernelGGL(mfma_f32_ws_kernel<SH>, grid, dim3(64 * kWsWaves), lds,
                     static_cast<hipStream_t>(stream), q, nblk, work);
  return check_launch("mfma_f32_ws_kernel");
}

// dispatch on SH = ceil((16 + 2r) / 4) over the radius classes DV = 2..6
typedef fobf_status (*F32WsLauncher)(const ImageParams&, int, float*, void*);
template <int... S>
constexpr std::array<F32WsLauncher, sizeof...(S)> f32_ws_table(std::integer_sequence<int, S...>) {
  return {&launch_f32_ws_sh<S + 5>...};
}
constexpr int kWsMinSH = 5;    // DV = 2
constexpr int kWsMaxSH = 24;   // DV = 6

template <typename OT>
fobf_status launch_staged_ws(const ImageParams& p, int DV, int nblk, float* work,
                             void* stream) {
  switch (DV) {
    case 2: return launch_staged_ws_dv<OT, 2>(p, nblk, work, stream);
    case 3: return launch_staged_ws_dv<OT, 3>(p, nblk, work, stream);
    case 4: return launch_staged_ws_dv<OT, 4>(p, nblk, work, stream);
    case 5: return launch_staged_ws_dv<OT, 5>(p, nblk, work, stream);
    case 6: return launch_staged_ws_dv<OT, 6>(p, nblk, work, stream);
    default: return fail(FOBF_EINTERNAL, "fobf_filter_ws: no workspace form for this radius");
  }
}

}  // namespace

// Tile height (16-row blocks) of the workspace forms, or 0 where they are
// not used: every precision (the LDS otherwise caps the tiles at 128 rows
// for float32 and single-word fp16, 96 for the two-word modes) at radius
// classes DV = 2..6 (eight strips; float32 from r = 14, above), and only
// when the image is tall enough
// for tiles of at least 8 blocks while still giving about one workgroup per
// compute unit (256 on the MI355X).  At most 32 blocks.  (Single-word fp16
// folds two frequencies per pass there; measured at 4096^2, K = 8 its
// workspace form takes 0.37 / 0.40 / 0.45 / 0.52 ms at theta = 5 / 8 / 10 /
// 12 against 0.47 / 0.53 / 0.62 / 0.80 ms for the LDS form.)
// Float32 takes the workspace form only from r = 14 on: below, its
// per-pass N/D round trips cost more than the LDS form's shorter tiles and
// per-wave trig (4096^2, K = 8: theta = 1 / 2 / 3 / 4 (r = 3..12) 0.72 /
// 0.73 / 0.91 / 0.96 ms against 0.59 / 0.64 / 0.87 / 0.93 for the LDS
// form; theta = 4.5 (r = 14) 0.966 / 0.968; theta = 5 1.00 / 1.05).  The
// staged precisions take it at every radius class it covers (fp16 0.33
// against 0.36 ms at theta = 2; the two-word ones within 1%).
constexpr int kF32WsMinR = 14;

int ws_nblk(const ImageParams& p, int prec) {
  if (prec < FOBF_FP32 || prec > FOBF_FP16X2_STAGE) return 0;
  const int DV = (MSTRIP + 2 * p.r + 15) / 16;
  if (DV < 2 || DV > 6 || p.H < 1 || p.W < 1) return 0;
  if (prec == FOBF_FP32 && p.r < kF32WsMinR) return 0;
  const long ntx = (p.W + kWsWaves * MSTRIP - 1) / (kWsWaves * MSTRIP);
  const long rows = (p.H + 15) / 16;
  const long nty_target = (256 + ntx - 1) / ntx;
  const long nblk = std::min<long>(32, (rows + nty_target - 1) / nty_target);
  return nblk >= 8 ? static_cast<int>(nblk) : 0;
}

size_t ws_bytes(const ImageParams& p, int prec) {
  const int nblk = ws_nblk(p, prec);
  if (nblk == 0) return 0;
  const size_t ntx = (p.W + kWsWaves * MSTRIP - 1) / (kWsWaves * MSTRIP);
  const size_t nty = (p.H + 16 * nblk - 1) / (16 * nblk);
  return sizeof(float) * ntx * nty * kWsWaves * 2 * 256 * static_cast<size_t>(nblk);
}

fobf_status launch_mfma_ws(const ImageParams& p0, int prec, float* work, void* stream) {
  const int nblk = ws_nblk(p0, prec);
  const int DV = (MSTRIP + 2 * p0.r + 15) / 16;
  if (nblk == 0) return fail(FOBF_EINTERNAL, "fobf_filter_ws: no workspace form");
  ImageParams p = p0;   // the workspace extent, for the debug-check build
  p.ws = work;
  p.ws_floats = static_cast<long long>(ws_bytes(p0, prec) / sizeof(float));
  if (prec == FOBF_FP32) {
    static const auto table =
        f32_ws_table(std::make_integer_sequence<int, kWsMaxSH - kWsMinSH + 1>{});
    const int SH = (MSTRIP + 2 * p.r + 3) / 4;
    if (SH < kWsMinSH || SH > kWsMaxSH)
      return fail(FOBF_EINTERNAL, "fobf_filter_ws: no workspace form for this radius");
    return table[SH - kWsMinSH](p, nblk, work, stream);
  }
  if (prec == FOBF_FP16_STAGE) return launch_staged_ws<_Float16>(p, DV, nblk, work, stream);
  if (prec == FOBF_BF16_STAGE) return launch_staged_ws<__bf16>(p, DV, nblk, work, stream);
  return launch_staged_ws<F16Pair>(p, DV, nblk, work, stream);
}

}  // namespace fobf
