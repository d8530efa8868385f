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
#include "fobf_batch_kern.h"

namespace fobf {

// float32 launchers: every radius class of the float32 body
BatchLauncher batch_launcher_f32(int cidx) {
  switch (cidx) {
    case 0: return launch_batch<FOBF_FP32, 2, 4>;
    case 1: return launch_batch<FOBF_FP32, 5, 5>;
    default: return launch_batch<FOBF_FP32, 6, 7>;
  }
}

namespace {
BatchLauncher launcher_for(int prec, int cidx) {
  return prec == FOBF_FP32 ? batch_launcher_f32(cidx) : batch_launcher_staged(prec, cidx);
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
  // a launch class with only a few tiles per workgroup slot runs them in a
  // few rounds, each as long as the longest tile's chain of blocks: cap the
  // tile height of all its jobs where that shortens rounds x chain (the
  // short requests of a serving batch; large batches keep their heights)
  for (int cls = 0; cls < MAX_LAUNCHES; ++cls) {
    const long slots = static_cast<long>(device_cus()) *
                       (cls % kRadiusClasses == 2 ? 1 : 2);
    int dvmax = 0;
    auto tiles = [&](int cap) {
      long t = 0;
      for (const Entry& e : es)
        if (e.cls == cls) {
          const int nb = std::min(e.b.nblk, cap);
          t += static_cast<long>(e.b.ntx) * ((e.b.p.H + 16 * nb - 1) / (16 * nb));
          dvmax = std::max(dvmax, e.b.dv);
        }
      return t;
    };
    const long t8 = tiles(BATCH_NBLK_MAX);
    if (t8 == 0 || t8 >= 4 * slots) continue;
    auto cost = [&](int cap) { return ((tiles(cap) + slots - 1) / slots) * (cap + dvmax - 1); };
    int cap = BATCH_NBLK_MAX;
    long best = cost(cap);
    for (int c = BATCH_NBLK_MAX - 1; c >= 1; --c)
      if (cost(c) < best) best = cost(c), cap = c;
    for (Entry& e : es)
      if (e.cls == cls && e.b.nblk > cap) {
        e.b.nblk = cap;
        e.b.nty = (e.b.p.H + 16 * cap - 1) / (16 * cap);
        e.cost = static_cast<double>(4 * e.b.p.K - 3) * (cap + e.b.dv - 1) * (2 * e.b.p.r + 1);
      }
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
