// Batched filtering: many images of different sizes, radii, orders and
// coefficients in one persistent launch.
//
// The host lays the jobs out in a device table, largest first, each with
// its range of global tile indices.  A grid sized to fill the machine once
// (CUs x resident workgroups) then loops: a workgroup takes the next tile
// index from a shared counter (atomicAdd), finds its job by binary search
// over the tile ranges, loads that job's tables into LDS (only when the job
// changes), and runs the same tile body as the single-image kernels.  Small
// and large images, and cheap and costly radii, so share the machine
// instead of serialising behind one another; every workgroup exits when the
// counter passes the last tile.
//
// One launch serves all jobs of one precision whose radius class fits the
// kernel: DV = ceil((16 + 2r) / 16) <= 4 (r <= 24), DV = 5 (r <= 32) or
// 6 <= DV <= 7 (r <= 48).
// The float32 body is the single-image kernel's tile body for the job's own
// step count (every SH of the class is instantiated), so a float32 batch
// image equals its single-image launch bit for bit; measured on the
// 256-image batch of uneven sizes and radii 6..24 this is also 5% faster
// than one body per class with its steps rounded up to 4 DV (9.7 vs
// 10.25 ms).
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
      f32_tile<S>(im, tx, ty, nblk, tbl, Bt, At, nd);                     \
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

template <int PREC>
BatchLauncher launcher_for_p(int cidx) {
  switch (cidx) {
    case 0: return launch_batch<PREC, 2, 4>;
    case 1: return launch_batch<PREC, 5, 5>;
    default: return launch_batch<PREC, 6, 7>;
  }
}

BatchLauncher launcher_for(int prec, int cidx) {
  switch (prec) {
    case FOBF_FP32: return launcher_for_p<FOBF_FP32>(cidx);
    case FOBF_FP16_STAGE: return launcher_for_p<FOBF_FP16_STAGE>(cidx);
    case FOBF_BF16_STAGE: return launcher_for_p<FOBF_BF16_STAGE>(cidx);
    default: return launcher_for_p<FOBF_FP16X2_STAGE>(cidx);
  }
}

}  // namespace

size_t batch_workspace_bytes(int n) {
  return COUNTER_BYTES * MAX_LAUNCHES + sizeof(BatchJob) * static_cast<size_t>(std::max(n, 0));
}

// c_dev (optional, n entries): device rows the jobs' coefficients are read
// from instead of the float32 copy in the job table (the server's
// device-resident coefficient cache).
fobf_status filter_batch_impl(const fobf_job* jobs, int n, void* d_work, size_t work_bytes,
                              void* stream, const float* const* c_dev) {
  if (n < 0) return fail(FOBF_EINVAL, "fobf_filter_batch: n < 0");
  if (n == 0) return FOBF_OK;
  if (!jobs) return fail(FOBF_EINVAL, "fobf_filter_batch: jobs is NULL");
  if (!d_work) return fail(FOBF_EINVAL, "fobf_filter_batch: workspace is NULL");
  if (work_bytes < batch_workspace_bytes(n))
    return fail(FOBF_EINVAL, "fobf_filter_batch: workspace too small");
  if (reinterpret_cast<uintptr_t>(d_work) % 256 != 0)
    return fail(FOBF_EINVAL, "fobf_filter_batch: workspace must be 256-byte aligned");
  struct Entry {
    BatchJob b;
    double cost;
    int cls;      // launch class: prec * kRadiusClasses + radius class
  };
  std::vector<Entry> es;
  es.reserve(n);
  int rerouted = -1;   // last job whose fp16 staging runs as two-word fp16
  for (int i = 0; i < n; ++i) {
    const fobf_job& j = jobs[i];
    fobf_status st = validate_filter(j.d_in, j.d_out, j.H, j.W, j.ld_in, j.ld_out, j.theta, j.K,
                                     j.T, j.c, j.prec, FOBF_ALGO_MFMA);
    if (st != FOBF_OK) {
      set_error("fobf_filter_batch: job " + std::to_string(i) + ": " + fobf_last_error());
      return st;
    }
    if (j.H == 0 || j.W == 0) continue;
    const int prec = effective_prec(j.prec, j.K, j.T, j.c);
    if (prec != j.prec) rerouted = i;
    Entry e;
    std::memset(&e.b, 0, sizeof(e.b));
    make_params(e.b.p, j.d_in, j.d_out, j.H, j.W, j.ld_in, j.ld_out, j.theta, j.K, j.T, j.c);
    e.b.p.c_dev = c_dev ? c_dev[i] : nullptr;
    const int r = e.b.p.r;
    e.b.dv = (16 + 2 * r + 15) / 16;
    e.b.nblk = std::min(batch_tile_blocks(prec, e.b.dv, j.H),
                        class_nblk_cap(prec, radius_class(e.b.dv)));
    e.b.ntx = (j.W + MWAVES * MSTRIP - 1) / (MWAVES * MSTRIP);
    e.b.nty = (j.H + 16 * e.b.nblk - 1) / (16 * e.b.nblk);
    // cost of one tile ~ channels x (halo'd rows) x band
    e.cost = static_cast<double>(4 * j.K - 3) * (e.b.nblk + e.b.dv - 1) * (2 * r + 1);
    e.cls = prec * kRadiusClasses + radius_class(e.b.dv);
    es.push_back(e);
  }
  // per class: largest tiles first (their tail is the hardest to hide)
  std::stable_sort(es.begin(), es.end(), [](const Entry& a, const Entry& b) {
    if (a.cls != b.cls) return a.cls < b.cls;
    return a.cost * a.b.ntx * a.b.nty > b.cost * b.b.ntx * b.b.nty;
  });
  std::vector<BatchJob> table(es.size());
  char* base = static_cast<char*>(d_work);
  int* counters = reinterpret_cast<int*>(base);
  BatchJob* d_table = reinterpret_cast<BatchJob*>(base + COUNTER_BYTES * MAX_LAUNCHES);
  struct Launch {
    int cls, first, count, total;
  };
  std::vector<Launch> launches;
  for (size_t i = 0; i < es.size();) {
    size_t k = i;
    int tiles = 0;
    while (k < es.size() && es[k].cls == es[i].cls) {
      table[k] = es[k].b;
      table[k].tile_begin = tiles;
      table[k].p.lds_bytes = static_cast<int>(
          class_lds_bytes(es[i].cls / kRadiusClasses, es[i].cls % kRadiusClasses));
      tiles += es[k].b.ntx * es[k].b.nty;
      ++k;
    }
    launches.push_back({es[i].cls, static_cast<int>(i), static_cast<int>(k - i), tiles});
    i = k;
  }
  fobf_status up = upload_async(d_table, table.data(), sizeof(BatchJob) * table.size(), stream);
  if (up != FOBF_OK) return up;
  for (const Launch& L : launches) {
    if (L.cls < 0 || L.cls >= MAX_LAUNCHES)
      return fail(FOBF_EINTERNAL, "fobf_filter_batch: launch class without a counter");
    BatchLauncher fn = launcher_for(L.cls / kRadiusClasses, L.cls % kRadiusClasses);
    int* ctr = reinterpret_cast<int*>(base + COUNTER_BYTES * L.cls);
    fobf_status st = fn(d_table + L.first, L.count, L.total, ctr, stream);
    if (st != FOBF_OK) return st;
  }
  (void)counters;
  if (rerouted >= 0)
    return prec_status(FOBF_FP16_STAGE, FOBF_FP16X2_STAGE,
                       ("fobf_filter_batch: job " + std::to_string(rerouted)).c_str());
  return FOBF_OK;
}

}  // namespace fobf

extern "C" size_t fobf_batch_workspace_size(int n) { return fobf::batch_workspace_bytes(n); }

extern "C" fobf_status fobf_filter_batch(const fobf_job* jobs, int n, void* d_work,
                                         size_t work_bytes, void* hip_stream) {
  return fobf::filter_batch_impl(jobs, n, d_work, work_bytes, hip_stream, nullptr);
}
