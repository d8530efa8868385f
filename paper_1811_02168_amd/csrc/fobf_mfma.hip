// Single-image launches of the matrix-core filter kernels (the device
// building blocks, and the description of the method, are in fobf_tiles.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <utility>

#include "fobf_tiles.h"

namespace fobf {

namespace {

template <int SH>
__global__ __launch_bounds__(MTHREADS, (SH <= 20 ? 2 : 1)) void mfma_f32_kernel(ImageParams p,
                                                                          int nblk) {
  constexpr int DV = (SH + 3) / 4;
  extern __shared__ float lds[];
  const int ntx = (p.W + MWAVES * MSTRIP - 1) / (MWAVES * MSTRIP);
  const int nty = (p.H + 16 * nblk - 1) / (16 * nblk);
  int tx, ty;
  if (!tile_of_block(blockIdx.x, gridDim.x, ntx, nty, &tx, &ty)) return;
  float* tbl = lds;
  float* Bt = lds + LDS_TABLE;
  float* At = Bt + 4 * DV * 64;
  float* nd = At + 4 * DV * 64;
  const Img im = FOBF_IMG(p);
  poison_lds(im);
  FOBF_LOAD_TABLES(p, tbl);
  __syncthreads();
  build_f32_tables<SH>(im, tbl, p.r, Bt, At);
  __syncthreads();
  f32_tile<SH, true>(im, tx, ty, nblk, tbl, Bt, At, nd);
}

template <typename OT, int DV>
__global__ __launch_bounds__((64 * staged_waves<OT, DV>())) void mfma_staged_kernel(ImageParams p,
                                                                            int nblk) {
  constexpr int NW = staged_waves<OT, DV>();
  extern __shared__ float lds[];
  const int ntx = (p.W + NW * MSTRIP - 1) / (NW * MSTRIP);
  const int nty = (p.H + 16 * nblk - 1) / (16 * nblk);
  int tx, ty;
  if (!tile_of_block(blockIdx.x, gridDim.x, ntx, nty, &tx, &ty)) return;
  float* tbl = lds;
  typename Stage<OT>::T* sbuf = reinterpret_cast<typename Stage<OT>::T*>(lds + LDS_TABLE);
  float* nd = lds + LDS_TABLE + staged_buf_bytes<OT, DV, NW>() / sizeof(float);
  const Img im = FOBF_IMG(p);
  poison_lds(im);
  FOBF_LOAD_TABLES(p, tbl);
  __syncthreads();
  staged_tile<OT, DV, NW>(im, tx, ty, nblk, tbl, sbuf, nd);
}

// ------------------------------------------------------------------ host --

template <int SH>
fobf_status launch_f32_sh(const ImageParams& p, int nblk, void* stream) {
  constexpr int DV = (SH + 3) / 4;
  static const bool once = (allow_big_lds(mfma_f32_kernel<SH>), true);
  (void)once;
  nblk = fill_nblk(p.H, p.W, nblk, MWAVES, SH <= 20 ? 2 : 1, DV);
  const size_t lds = sizeof(float) * (LDS_TABLE + 8 * DV * 64 +
                                      static_cast<size_t>(MWAVES) * 2 * nblk * 256);
  dim3 grid(padded_blocks(p, nblk));
  ImageParams q = p;
  q.lds_bytes = static_cast<int>(lds);
  hipLaunchKernelGGL(mfma_f32_kernel<SH>, grid, dim3(MTHREADS), lds,
                     static_cast<hipStream_t>(stream), q, nblk);
  return check_launch("mfma_f32_kernel");
}

// dispatch on SH = ceil((16 + 2r) / 4), 5 .. 4 + FOBF_RMAX / 2
typedef fobf_status (*F32Launcher)(const ImageParams&, int, void*);
template <int... S>
constexpr std::array<F32Launcher, sizeof...(S)> f32_table(std::integer_sequence<int, S...>) {
  return {&launch_f32_sh<S + 5>...};
}
constexpr int kMinSH = 5;
constexpr int kMaxSH = (MSTRIP + 2 * FOBF_RMAX + 3) / 4;

template <typename OT, int DV>
fobf_status launch_staged_dv(const ImageParams& p, int nblk, void* stream) {
  static const bool once = (allow_big_lds(mfma_staged_kernel<OT, DV>), true);
  (void)once;
  constexpr int NW = staged_waves<OT, DV>();
  // the tallest tile whose per-wave N and D still fit next to the staging
  constexpr size_t fixed = sizeof(float) * LDS_TABLE + staged_buf_bytes<OT, DV, NW>();
  constexpr int cap = static_cast<int>((160 * 1024 - fixed) / (sizeof(float) * NW * 2 * 256));
  nblk = fill_nblk(p.H, p.W, std::min(nblk, cap), NW, 1, DV);
  const size_t lds = fixed + sizeof(float) * NW * 2 * nblk * 256;
  dim3 grid(padded_blocks(p, nblk, NW));
  ImageParams q = p;
  q.lds_bytes = static_cast<int>(lds);
  hipLaunchKernelGGL((mfma_staged_kernel<OT, DV>), grid, dim3(64 * NW), lds,
                     static_cast<hipStream_t>(stream), q, nblk);
  return check_launch("mfma_staged_kernel");
}

template <typename OT>
fobf_status launch_staged(const ImageParams& p, int DV, int nblk, void* stream) {
  switch (DV) {
    case 2: return launch_staged_dv<OT, 2>(p, nblk, stream);
    case 3: return launch_staged_dv<OT, 3>(p, nblk, stream);
    case 4: return launch_staged_dv<OT, 4>(p, nblk, stream);
    case 5: return launch_staged_dv<OT, 5>(p, nblk, stream);
    case 6: return launch_staged_dv<OT, 6>(p, nblk, stream);
    case 7: return launch_staged_dv<OT, 7>(p, nblk, stream);
    default: return fail(FOBF_EINVAL, "fobf_filter: radius out of range for the MFMA path");
  }
}

}  // namespace

fobf_status launch_mfma(const ImageParams& p, int prec, int nblk, void* stream) {
  const int DV = (MSTRIP + 2 * p.r + 15) / 16;
  if (nblk < 1 || nblk > 16) return fail(FOBF_EINVAL, "fobf_filter: tile height out of range");
  if (prec == FOBF_FP16_STAGE) return launch_staged<_Float16>(p, DV, nblk, stream);
  if (prec == FOBF_BF16_STAGE) return launch_staged<__bf16>(p, DV, nblk, stream);
  if (prec == FOBF_FP16X2_STAGE) return launch_staged<F16Pair>(p, DV, nblk, stream);
  static const auto table = f32_table(std::make_integer_sequence<int, kMaxSH - kMinSH + 1>{});
  const int SH = (MSTRIP + 2 * p.r + 3) / 4;
  if (SH < kMinSH || SH > kMaxSH)
    return fail(FOBF_EINVAL, "fobf_filter: radius out of range for the MFMA path");
  return table[SH - kMinSH](p, nblk, stream);
}



}  // namespace fobf
