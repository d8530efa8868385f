// Persistent batch kernel shared by the batch translation units: the job
// table entry, the kernel (an atomic tile queue over the tile bodies of
// fobf_tiles.h), its LDS budget per launch class and its launcher.  The
// float32 and the staged instantiations are compiled in separate units
// (fobf_batch.hip, fobf_batch_staged.hip), each exporting the launchers of
// its precisions.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "fobf_tiles.h"

namespace fobf {

struct BatchJob {
  ImageParams p;
  int tile_begin;   // first global tile index of this job
  int ntx, nty;     // tiles across / down
  int nblk;         // 16-row blocks per tile (tile height 16 * nblk)
  int dv;           // ceil((16 + 2r) / 16)
  int pad_[3];
};

namespace {

constexpr int BATCH_NBLK_MAX = 8;
constexpr size_t COUNTER_BYTES = 256;   // one counter per launch, own line
// Radius classes of the batch launches (DV = ceil((16 + 2r)/16)): r <= 24,
// 24 < r <= 32, 32 < r <= 48.  One counter per launch class: each
// precision x each radius class.
constexpr int kRadiusClasses = 3;
constexpr int radius_class(int dv) { return dv <= 4 ? 0 : (dv == 5 ? 1 : 2); }
constexpr int MAX_LAUNCHES = kRadiusClasses * kNumPrecisions;

__global__ void reset_counter(int* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0;
}

// Two workgroups per CU (256 VGPRs per lane, half the LDS each) for the
// radius classes whose tile bodies fit that budget (DV <= 5); one for the
// largest radii, which need more registers.
template <int DVHI>
constexpr int batch_min_blocks() { return DVHI <= 5 ? 2 : 1; }

template <int PREC, int DVLO, int DVHI>
__global__ __launch_bounds__(MTHREADS, batch_min_blocks<DVHI>()) void batch_kernel(
    const BatchJob* __restrict__ jobs,
                                                            int njobs, int total,
                                                            int* __restrict__ counter) {
  extern __shared__ float lds[];
  __shared__ int s_tile;
  float* tbl = lds;
  int cur = -1;
  if (njobs > 0) poison_lds(FOBF_IMG(jobs[0].p));
  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1);
    __syncthreads();
    const int t = s_tile;
    if (t >= total) break;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (jobs[mid].tile_begin <= t) lo = mid; else hi = mid - 1;
    }
    const BatchJob* J = jobs + lo;
    const int lt = t - J->tile_begin;
    const int ty = lt / J->ntx;
    const int tx = lt - ty * J->ntx;
    const int nblk = J->nblk;
    const int dv = J->dv;
    const Img im = FOBF_IMG(J->p);
    FOBF_CHK(im, lt >= 0 && ty < J->nty && dv >= DVLO && dv <= DVHI, FOBF_CHECK_TILE);
    // check builds: what the previous tile left in the LDS is poisoned
    // again (the tables stay while the job does)
    poison_lds(im, sizeof(float) * LDS_TABLE);
    if (lo != cur) {
      FOBF_LOAD_TABLES(J->p, tbl);
      cur = lo;
    }
    __syncthreads();
    if constexpr (PREC == FOBF_FP32) {
      float* Bt = lds + LDS_TABLE;
      float* At = Bt + 4 * DVHI * 64;
      float* nd = At + 4 * DVHI * 64;
      // the job's own step count SH = ceil((16 + 2r) / 4): the tile body
      // of the single-image kernel, bit for bit
      switch ((MSTRIP + 2 * im.r + 3) / 4) {
#define FOBF_F32_CASE(S)                                                  \
  case S:                                                                 \
    if constexpr ((S + 3) / 4 >= DVLO && (S + 3) / 4 <= DVHI) {           \
      build_f32_tables<S>(im, tbl, im.r, Bt, At);                         \
      __syncthreads();                                                    \
      f32_tile<S, true>(im, tx, ty, nblk, tbl, Bt, At, nd);               \
    }                                                                     \
    break;
#define FOBF_F32_CASES(D) \
  FOBF_F32_CASE(4 * D - 3) FOBF_F32_CASE(4 * D - 2) FOBF_F32_CASE(4 * D - 1) FOBF_F32_CASE(4 * D)
        FOBF_F32_CASES(2)
        FOBF_F32_CASES(3)
        FOBF_F32_CASES(4)
        FOBF_F32_CASES(5)
        FOBF_F32_CASES(6)
        FOBF_F32_CASES(7)
#undef FOBF_F32_CASES
#undef FOBF_F32_CASE
        default: break;
      }
    } else {
      typedef typename std::conditional<
          PREC == FOBF_FP16_STAGE, _Float16,
          typename std::conditional<PREC == FOBF_BF16_STAGE, __bf16, F16Pair>::type>::type OT;
      typename Stage<OT>::T* sbuf = reinterpret_cast<typename Stage<OT>::T*>(lds + LDS_TABLE);
      float* nd = lds + LDS_TABLE + staged_buf_bytes<OT, DVHI, MWAVES>() / sizeof(float);
      switch (dv) {
#define FOBF_ST_CASE(D)                                               \
  case D:                                                             \
    if constexpr (D >= DVLO && D <= DVHI) staged_tile<OT, D, MWAVES>(im, tx, ty, nblk, tbl, sbuf, nd); \
    break;
        FOBF_ST_CASE(2)
        FOBF_ST_CASE(3)
        FOBF_ST_CASE(4)
        FOBF_ST_CASE(5)
        FOBF_ST_CASE(6)
        FOBF_ST_CASE(7)
#undef FOBF_ST_CASE
        default: break;
      }
    }
    __syncthreads();   // tile done before s_tile and the tables are rewritten
  }
}

// LDS of a batch launch besides the per-wave N/D blocks
template <int PREC, int DVHI>
constexpr size_t batch_fixed_lds() {
  if (PREC == FOBF_FP32) return sizeof(float) * (LDS_TABLE + 8 * DVHI * 64);
  if (PREC == FOBF_FP16_STAGE) return sizeof(float) * LDS_TABLE + staged_buf_bytes<_Float16, DVHI, MWAVES>();
  if (PREC == FOBF_BF16_STAGE) return sizeof(float) * LDS_TABLE + staged_buf_bytes<__bf16, DVHI, MWAVES>();
  return sizeof(float) * LDS_TABLE + staged_buf_bytes<F16Pair, DVHI, MWAVES>();
}

// tallest tile (16-row blocks) whose N/D still fits the LDS share of one
// workgroup (160 KB over the workgroups per CU the class is built for)
template <int PREC, int DVHI>
constexpr int batch_nblk_cap() {
  constexpr size_t room =
      160 * 1024 / batch_min_blocks<DVHI>() - 256 - batch_fixed_lds<PREC, DVHI>();
  constexpr int nb = static_cast<int>(room / (sizeof(float) * MWAVES * 2 * 256));
  return nb < BATCH_NBLK_MAX ? nb : BATCH_NBLK_MAX;
}

template <int PREC, int DVHI>
size_t batch_lds_bytes() {
  return batch_fixed_lds<PREC, DVHI>() +
         sizeof(float) * MWAVES * 2 * batch_nblk_cap<PREC, DVHI>() * 256;
}

// dynamic LDS bytes of a launch class (precision, radius class)
template <int PREC>
size_t class_lds_bytes_p(int cidx) {
  switch (cidx) {
    case 0: return batch_lds_bytes<PREC, 4>();
    case 1: return batch_lds_bytes<PREC, 5>();
    default: return batch_lds_bytes<PREC, 7>();
  }
}

size_t class_lds_bytes(int prec, int cidx) {
  switch (prec) {
    case FOBF_FP32: return class_lds_bytes_p<FOBF_FP32>(cidx);
    case FOBF_FP16_STAGE: return class_lds_bytes_p<FOBF_FP16_STAGE>(cidx);
    case FOBF_BF16_STAGE: return class_lds_bytes_p<FOBF_BF16_STAGE>(cidx);
    default: return class_lds_bytes_p<FOBF_FP16X2_STAGE>(cidx);
  }
}

template <int PREC, int DVLO, int DVHI>
fobf_status launch_batch(const BatchJob* d_jobs, int njobs, int total, int* d_counter,
                         void* stream) {
  auto kern = batch_kernel<PREC, DVLO, DVHI>;
  const size_t lds = batch_lds_bytes<PREC, DVHI>();
  static int grid = 0;
  static std::once_flag once;
  std::call_once(once, [&]() {
    // exactly the dynamic size (the kernel also holds a little static LDS)
    hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                        hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    int dev = 0, cus = 0, occ = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, MTHREADS, lds);
    grid = std::max(1, cus) * std::max(1, occ);
  });
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, s, d_counter);
  const int g = std::max(1, std::min(grid, total));
  hipLaunchKernelGGL(kern, dim3(g), dim3(MTHREADS), lds, s, d_jobs, njobs, total, d_counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(FOBF_EHIP, std::string("batch_kernel launch: ") + hipGetErrorString(e));
  return FOBF_OK;
}

typedef fobf_status (*BatchLauncher)(const BatchJob*, int, int, int*, void*);

// per (precision, radius class): tile-height cap and launcher
template <int PREC>
int class_nblk_cap_p(int cidx) {
  switch (cidx) {
    case 0: return batch_nblk_cap<PREC, 4>();
    case 1: return batch_nblk_cap<PREC, 5>();
    default: return batch_nblk_cap<PREC, 7>();
  }
}

int class_nblk_cap(int prec, int cidx) {
  switch (prec) {
    case FOBF_FP32: return class_nblk_cap_p<FOBF_FP32>(cidx);
    case FOBF_FP16_STAGE: return class_nblk_cap_p<FOBF_FP16_STAGE>(cidx);
    case FOBF_BF16_STAGE: return class_nblk_cap_p<FOBF_BF16_STAGE>(cidx);
    default: return class_nblk_cap_p<FOBF_FP16X2_STAGE>(cidx);
  }
}

}  // namespace

// Launchers of the batch kernel per launch class (radius class 0..2):
// float32 (fobf_batch.hip) and the staged precisions (fobf_batch_staged.hip).
BatchLauncher batch_launcher_f32(int cidx);
BatchLauncher batch_launcher_staged(int prec, int cidx);

}  // namespace fobf
