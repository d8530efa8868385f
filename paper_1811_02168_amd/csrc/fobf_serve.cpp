// Continuous-batching server for the Fourier bilateral filter.
//
// submit() may be called from any thread at any time; it validates the
// request, stamps it and queues it.  One scheduler thread admits queued
// requests in arrival order while the number in flight and their device
// bytes (below) fit the configured limits, merges up to
// max_batch admitted requests into one batch, and issues the batch on the
// least loaded of a few HIP streams ("lanes": the one with the fewest
// pixels in flight, so that a small request does not wait in stream order
// behind a large one): per request a stream-ordered device
// allocation and the host-to-device copy, then ONE persistent batched
// launch for all of them (fobf_filter_batch's kernel), then the copies back
// and stream-ordered frees.  A request large enough for the workspace form
// of the filter (tall tiles, N and D in a workspace: the fobf_filter_ws
// condition) runs that form instead, one launch of its own on the same
// lane after the batch, its workspace drawn from the same pool.  A host callback at the end of each batch marks
// its requests done and returns their bytes to the budget, which lets the
// scheduler admit more: requests that arrive while others are on the
// device join the next batch as soon as memory frees up, and batches on
// different lanes overlap (copies of one with the kernel of another).
//
// Coefficients are fitted on the host (float64, cached by (R, sigma, K))
// by a small pool of fit threads -- the period by a local search started
// from the periods of already fitted neighbouring sigmas -- so that a request whose (sigma, K) has not
// been seen yet never holds up the admission of requests whose
// coefficients are ready: the scheduler admits, in arrival order, the
// queued requests whose fit has finished.  Each distinct fit is uploaded
// once into a device-resident table that the batched kernel reads them
// from.  Ordering rule: the upload of a row is enqueued on the lane of the
// first batch that uses it, followed by an event; every later batch that
// reads the row, on whatever lane, waits for that event on its own lane
// before its kernel (until the event has been seen complete), so no
// kernel can read a row before its bytes have landed.
//
// Device memory: request images, each batch's job table and the workspace
// of a request that runs the workspace form come from a memory pool private
// to the server whose release threshold is the HBM budget (the process's
// default pool is left untouched); each request is charged its two images
// plus the larger of one batch-workspace share and its own workspace.
//
// Host image buffers should be pinned (hipHostMalloc, or torch's
// pin_memory) for the copies to be asynchronous; pageable buffers work but
// make the scheduler wait for each copy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "fobf_internal.h"

namespace fobf {
fobf_status filter_batch_impl(const fobf_job* jobs, int n, void* d_work, size_t work_bytes,
                              void* stream, const float* const* c_dev);
size_t batch_workspace_bytes(int n);
}  // namespace fobf

using namespace fobf;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

typedef std::tuple<int, uint64_t, int> CoefKey;   // (R, sigma bits, K)

struct Req {
  uint64_t ticket;
  CoefKey key;
  fobf_request r;
  fobf_result res;
  bool done = false;
  size_t bytes = 0;
  float* d_in = nullptr;
  float* d_out = nullptr;
  int T = 0;
  const float* c_dev = nullptr;
  double c[FOBF_KMAX];
};

struct Batch;

constexpr int kLanes = 3;
constexpr int kFitThreads = 2;
constexpr int kCoefSlots = 4096;

}  // namespace

struct fobf_server {
  fobf_serve_cfg cfg{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work;
  std::condition_variable cv_done;
  std::deque<Req*> pending;
  std::unordered_map<uint64_t, Req*> reqs;
  uint64_t next_ticket = 1;
  size_t bytes_inflight = 0;
  int n_inflight = 0;
  int batches_running = 0;
  bool stop = false;
  int inject = 0;
  std::thread worker;
  std::thread fitters[kFitThreads];
  std::condition_variable cv_fit;
  std::deque<CoefKey> fit_queue;
  hipStream_t lanes[kLanes] = {};
  // pixels of the batches issued on each lane and not yet done (guarded
  // by mu): a new batch goes to the lane with the least outstanding work,
  // so that small requests do not queue behind a large one in stream order
  double lane_pixels[kLanes] = {};
  // fit cache: (R, sigma bits, K) -> (state, T, c, device row).  Guarded
  // by mu; only the scheduler thread uploads rows.
  enum CoefState { kFitting, kReady, kFailed };
  struct Coef {
    CoefState state;
    fobf_status status;
    int T;
    double c[FOBF_KMAX];
    const float* row;
    hipEvent_t uploaded;   // recorded after the row's upload (or null)
    bool landed;           // the event has been seen complete
  };
  std::map<CoefKey, Coef> coef;
  float* d_coef = nullptr;
  int coef_used = 0;
  hipMemPool_t pool = nullptr;   // private pool for request buffers
  fobf_serve_stats stats{};
};

namespace {

struct Batch {
  fobf_server* s;
  std::vector<Req*> reqs;
  int lane;
  double pixels;   // the batch's share of lane_pixels[lane]
};

// Runs on a HIP runtime thread when a batch's stream reaches its end: no
// HIP calls here, only bookkeeping under the server lock.
void batch_done(void* arg) {
  Batch* b = static_cast<Batch*>(arg);
  fobf_server* s = b->s;
  const double t = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (Req* q : b->reqs) {
      q->res.t_done = t;
      if (q->res.status == FOBF_EBUSY) q->res.status = FOBF_OK;
      q->done = true;
      s->bytes_inflight -= q->bytes;
      s->n_inflight -= 1;
      s->stats.completed += 1;
      if (q->res.status != FOBF_OK) s->stats.failed += 1;
    }
    s->batches_running -= 1;
    s->lane_pixels[b->lane] -= b->pixels;
  }
  s->cv_done.notify_all();
  s->cv_work.notify_all();
  delete b;
}

// Completes requests that never reached the device (caller holds no lock).
void finish_now(fobf_server* s, const std::vector<Req*>& qs, fobf_status st) {
  const double t = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (Req* q : qs) {
      q->res.status = st;
      q->res.t_done = t;
      q->done = true;
      s->bytes_inflight -= q->bytes;
      s->n_inflight -= 1;
      s->stats.completed += 1;
      s->stats.failed += 1;
    }
  }
  s->cv_done.notify_all();
  s->cv_work.notify_all();
}

// Stream-ordered device allocation from the server's private pool (or the
// device's default pool where a private one could not be created).
hipError_t device_alloc(fobf_server* s, void** p, size_t bytes, hipStream_t st) {
  *p = nullptr;
  if (s->pool) return hipMallocFromPoolAsync(p, bytes, s->pool, st);
  return hipMallocAsync(p, bytes, st);
}

// Device bytes a request is charged against the budget: its input and
// output images plus the larger of one batch-workspace share (job-table
// entry and the launch counters) and the N/D workspace of the workspace
// form (zero where that form is not used; the staged precisions share one
// rule, so an fp16 request run as two-word fp16 needs the same), so that
// every batch's and every workspace launch's memory is covered.
size_t request_bytes(int H, int W, double theta, int prec) {
  ImageParams p;
  std::memset(&p, 0, sizeof(p));
  p.H = H;
  p.W = W;
  p.r = spatial_radius(theta);
  return 2 * sizeof(float) * static_cast<size_t>(H) * W +
         std::max(batch_workspace_bytes(1), ws_bytes(p, prec));
}

// Coefficients of an admitted request (its fit has finished): the first
// use of a fit uploads its float32 row into the device table.  Scheduler
// thread only.
fobf_status coefficients(fobf_server* s, Req* q, hipStream_t st) {
  fobf_server::Coef e;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    e = s->coef.at(q->key);
  }
  if (e.state == fobf_server::kFailed) return fail(e.status, "fobf_serve: coefficient fit failed");
  if (!e.row && s->coef_used < kCoefSlots) {
    float row[FOBF_KMAX];
    for (int k = 0; k < FOBF_KMAX; ++k) row[k] = k < q->r.K ? static_cast<float>(e.c[k]) : 0.f;
    float* dst = s->d_coef + static_cast<size_t>(s->coef_used) * FOBF_KMAX;
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
      return fail(FOBF_EHIP, "fobf_serve: event creation failed");
    fobf_status up = upload_async(dst, row, sizeof(row), st);
    if (up == FOBF_OK && hipEventRecord(ev, st) != hipSuccess)
      up = fail(FOBF_EHIP, "fobf_serve: event record failed");
    if (up != FOBF_OK) {
      hipEventDestroy(ev);
      return up;
    }
    s->coef_used += 1;
    e.row = dst;
    e.uploaded = ev;
    e.landed = false;
    std::lock_guard<std::mutex> lk(s->mu);
    fobf_server::Coef& m = s->coef.at(q->key);
    m.row = dst;
    m.uploaded = ev;
    m.landed = false;
  } else if (e.row && e.uploaded && !e.landed) {
    // the row was uploaded by an earlier batch, possibly on another lane:
    // order this lane after the upload unless it is known to have landed
    const hipError_t qe = hipEventQuery(e.uploaded);
    if (qe == hipSuccess) {
      std::lock_guard<std::mutex> lk(s->mu);
      s->coef.at(q->key).landed = true;
    } else if (hipStreamWaitEvent(st, e.uploaded, 0) != hipSuccess) {
      return fail(FOBF_EHIP, "fobf_serve: stream wait on the coefficient upload failed");
    }
  }
  q->T = e.T;
  std::memcpy(q->c, e.c, sizeof(q->c));
  q->c_dev = e.row;
  return FOBF_OK;
}

// Start of the period search for a new key: the periods already fitted
// for the same (R, K) at the nearest sigma below and above, interpolated
// linearly in sigma (the optimal period varies smoothly with sigma, Sec. II
// after Algorithm 1), or the one neighbour there is, or 0 (the search then
// starts at T = R).  Caller holds s->mu.
int warm_period(fobf_server* s, const CoefKey& key, double sigma) {
  const int R = std::get<0>(key), K = std::get<2>(key);
  double slo = -1.0, shi = -1.0;
  int tlo = 0, thi = 0;
  for (const auto& kv : s->coef) {
    if (std::get<0>(kv.first) != R || std::get<2>(kv.first) != K) continue;
    if (kv.second.state != fobf_server::kReady) continue;
    double sg;
    const uint64_t b = std::get<1>(kv.first);
    std::memcpy(&sg, &b, sizeof(sg));
    if (sg <= sigma && (slo < 0.0 || sg > slo)) {
      slo = sg;
      tlo = kv.second.T;
    }
    if (sg >= sigma && (shi < 0.0 || sg < shi)) {
      shi = sg;
      thi = kv.second.T;
    }
  }
  if (slo >= 0.0 && shi >= 0.0 && shi > slo)
    return static_cast<int>(std::lround(tlo + (thi - tlo) * (sigma - slo) / (shi - slo)));
  if (slo >= 0.0) return tlo;
  if (shi >= 0.0) return thi;
  return 0;
}

// Fit threads: solve queued (R, sigma, K) keys on the host (the period by
// a local search from warm_period, fobf_fit_warm) and mark them ready (or
// failed), then wake the scheduler.
void fitter_main(fobf_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_fit.wait(lk, [&]() { return s->stop || !s->fit_queue.empty(); });
    if (s->stop) return;
    const CoefKey key = s->fit_queue.front();
    s->fit_queue.pop_front();
    double sigma;
    const uint64_t sb = std::get<1>(key);
    std::memcpy(&sigma, &sb, sizeof(sigma));
    const int T0 = warm_period(s, key, sigma);
    lk.unlock();
    fobf_coef fc;
    const fobf_status st =
        fobf_fit_warm(std::get<0>(key), sigma, std::get<2>(key), s->cfg.eps, 0, T0, &fc);
    lk.lock();
    fobf_server::Coef& e = s->coef.at(key);
    if (st == FOBF_OK || st == FOBF_WARN_TOL) {
      e.state = fobf_server::kReady;
      e.T = fc.T;
      for (int k = 0; k < std::get<2>(key); ++k) e.c[k] = fc.c[k];
    } else {
      e.state = fobf_server::kFailed;
      e.status = st;
    }
    s->cv_work.notify_all();
  }
}

void submit_batch(fobf_server* s, std::vector<Req*>& adm) {
  // the lane with the least outstanding work (the copies, which dominate a
  // request's device time, scale with its pixels); only this thread issues
  int lane = 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (int i = 1; i < kLanes; ++i)
      if (s->lane_pixels[i] < s->lane_pixels[lane]) lane = i;
  }
  hipStream_t st = s->lanes[lane];
  bool inject = false;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->inject > 0) {
      s->inject -= 1;
      inject = true;
    }
  }
  if (inject) {
    set_error("fobf_serve: injected device submission failure");
    finish_now(s, adm, FOBF_EHIP);
    return;
  }
  const double t0 = now_s();
  std::vector<Req*> ok;
  std::vector<Req*> bad;
  std::vector<fobf_job> jobs;
  std::vector<const float*> cdev;
  struct Tall {
    Req* q;
    ImageParams p;
    int prec;
  };
  std::vector<Tall> tall;   // requests that run the workspace form
  for (Req* q : adm) {
    q->res.t_start = t0;
    fobf_status cs = coefficients(s, q, st);
    if (cs != FOBF_OK) {
      q->res.status = cs;
      bad.push_back(q);
      continue;
    }
    const size_t img = sizeof(float) * static_cast<size_t>(q->r.H) * q->r.W;
    if (device_alloc(s, reinterpret_cast<void**>(&q->d_in), img, st) != hipSuccess ||
        device_alloc(s, reinterpret_cast<void**>(&q->d_out), img, st) != hipSuccess) {
      if (q->d_in) hipFreeAsync(q->d_in, st);
      q->d_in = q->d_out = nullptr;
      q->res.status = FOBF_ENOMEM;
      bad.push_back(q);
      continue;
    }
    const size_t row = sizeof(float) * q->r.W;
    if (hipMemcpy2DAsync(q->d_in, row, q->r.h_in, sizeof(float) * q->r.ld_in, row, q->r.H,
                         hipMemcpyHostToDevice, st) != hipSuccess) {
      hipFreeAsync(q->d_in, st);
      hipFreeAsync(q->d_out, st);
      q->d_in = q->d_out = nullptr;
      set_error("fobf_serve: host-to-device copy failed");
      q->res.status = FOBF_EHIP;
      bad.push_back(q);
      continue;
    }
    fobf_job j{};
    j.d_in = q->d_in;
    j.d_out = q->d_out;
    j.H = q->r.H;
    j.W = q->r.W;
    j.ld_in = j.ld_out = q->r.W;
    j.theta = q->r.theta;
    j.K = q->r.K;
    j.T = q->T;
    j.prec = effective_prec(q->r.prec, q->r.K, q->T, q->c);
    for (int k = 0; k < q->r.K; ++k) j.c[k] = q->c[k];
    q->res.prec = j.prec;
    q->res.T = q->T;
    ok.push_back(q);
    Tall t{q, {}, j.prec};
    make_params(t.p, j.d_in, j.d_out, j.H, j.W, j.ld_in, j.ld_out, j.theta, j.K, j.T, q->c);
    t.p.c_dev = q->c_dev;
    if (ws_nblk(t.p, j.prec) > 0) {
      tall.push_back(t);
      continue;
    }
    jobs.push_back(j);
    cdev.push_back(q->c_dev);
  }
  for (Req* q : bad) finish_now(s, {q}, q->res.status);
  if (ok.empty()) return;
  void* ws = nullptr;
  fobf_status st_b = FOBF_OK;
  if (!jobs.empty()) {
    const size_t wsb = batch_workspace_bytes(static_cast<int>(jobs.size()));
    if (device_alloc(s, &ws, wsb, st) != hipSuccess) {
      st_b = fail(FOBF_ENOMEM, "fobf_serve: workspace allocation failed");
    } else {
      st_b = filter_batch_impl(jobs.data(), static_cast<int>(jobs.size()), ws, wsb, st,
                               cdev.data());
    }
  }
  // the batch's status belongs to its requests; a workspace-form request
  // carries its own
  std::unordered_map<Req*, fobf_status> own;
  for (Tall& t : tall) {
    void* w = nullptr;
    fobf_status st_t;
    if (device_alloc(s, &w, ws_bytes(t.p, t.prec), st) != hipSuccess) {
      st_t = fail(FOBF_ENOMEM, "fobf_serve: workspace allocation failed");
    } else {
      st_t = launch_mfma_ws(t.p, t.prec, static_cast<float*>(w), st);
      hipFreeAsync(w, st);
    }
    own[t.q] = st_t;
  }
  for (Req* q : ok) {
    const auto it = own.find(q);
    const fobf_status st_q = it != own.end() ? it->second : st_b;
    if (st_q == FOBF_OK) {
      const size_t row = sizeof(float) * q->r.W;
      if (hipMemcpy2DAsync(q->r.h_out, sizeof(float) * q->r.ld_out, q->d_out, row, row,
                           q->r.H, hipMemcpyDeviceToHost, st) != hipSuccess) {
        set_error("fobf_serve: device-to-host copy failed");
        q->res.status = FOBF_EHIP;
      }
    } else {
      q->res.status = st_q;
    }
    hipFreeAsync(q->d_in, st);
    hipFreeAsync(q->d_out, st);
  }
  if (ws) hipFreeAsync(ws, st);
  double pixels = 0.0;
  for (Req* q : ok) pixels += static_cast<double>(q->r.H) * q->r.W;
  Batch* b = new Batch{s, ok, lane, pixels};
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->lane_pixels[lane] += pixels;
    s->batches_running += 1;
    s->stats.batches += 1;
    s->stats.coef_entries = s->coef_used;
  }
  if (hipLaunchHostFunc(st, batch_done, b) != hipSuccess) {
    // no completion callback: wait here, then complete
    hipStreamSynchronize(st);
    batch_done(b);
  }
}

void worker_main(fobf_server* s) {
  hipSetDevice(s->device);
  for (;;) {
    std::vector<Req*> adm;
    std::vector<Req*> cancelled;
    std::vector<Req*> timed_out;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      // the first queued request whose fit has finished, if the limits let
      // it in (requests still waiting for a fit are passed over)
      auto next_ready = [&]() -> std::deque<Req*>::iterator {
        if (s->n_inflight >= s->cfg.max_inflight) return s->pending.end();
        for (auto it = s->pending.begin(); it != s->pending.end(); ++it) {
          if (s->coef.at((*it)->key).state == fobf_server::kFitting) continue;
          if (s->bytes_inflight + (*it)->bytes <= s->cfg.hbm_budget_bytes) return it;
          return s->pending.end();
        }
        return s->pending.end();
      };
      auto admissible = [&]() { return next_ready() != s->pending.end(); };
      // queued requests past their admission deadline, and the earliest
      // deadline still ahead (infinity when none)
      auto deadline = [](const Req* q) {
        return q->r.deadline_s > 0.0 ? q->res.t_submit + q->r.deadline_s : INFINITY;
      };
      auto expired_any = [&](double t) {
        for (const Req* q : s->pending)
          if (deadline(q) <= t) return true;
        return false;
      };
      for (;;) {
        if (s->stop || admissible() || expired_any(now_s())) break;
        double next = INFINITY;
        for (const Req* q : s->pending) next = std::min(next, deadline(q));
        if (next == INFINITY) {
          s->cv_work.wait(lk);
        } else {
          s->cv_work.wait_for(lk, std::chrono::duration<double>(std::max(0.0, next - now_s())));
        }
      }
      {
        const double t = now_s();
        for (auto it = s->pending.begin(); it != s->pending.end();) {
          if (deadline(*it) <= t) {
            timed_out.push_back(*it);
            it = s->pending.erase(it);
          } else {
            ++it;
          }
        }
      }
      if (s->stop) {
        while (!s->pending.empty()) {
          cancelled.push_back(s->pending.front());
          s->pending.pop_front();
        }
      } else {
        for (auto it = next_ready(); it != s->pending.end() &&
                                     static_cast<int>(adm.size()) < s->cfg.max_batch;
             it = next_ready()) {
          Req* q = *it;
          s->pending.erase(it);
          s->n_inflight += 1;
          s->bytes_inflight += q->bytes;
          s->stats.peak_inflight = std::max(s->stats.peak_inflight, s->n_inflight);
          s->stats.peak_bytes_inflight = std::max(s->stats.peak_bytes_inflight, s->bytes_inflight);
          q->res.t_admit = now_s();
          adm.push_back(q);
        }
      }
    }
    if (!cancelled.empty() || !timed_out.empty()) {
      const double t = now_s();
      {
        std::lock_guard<std::mutex> lk(s->mu);
        for (Req* q : cancelled) {
          q->res.status = FOBF_ECANCELED;
          q->res.t_done = t;
          q->done = true;
        }
        for (Req* q : timed_out) {
          q->res.status = FOBF_ETIMEDOUT;
          q->res.t_done = t;
          q->done = true;
          s->stats.completed += 1;
          s->stats.failed += 1;
        }
      }
      s->cv_done.notify_all();
    }
    if (!adm.empty()) submit_batch(s, adm);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->stop && s->pending.empty()) break;
    }
  }
  // drain: every batch on the device finishes before the server goes away
  for (int i = 0; i < kLanes; ++i) hipStreamSynchronize(s->lanes[i]);
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&]() { return s->batches_running == 0; });
}

}  // namespace

extern "C" fobf_status fobf_serve_create(const fobf_serve_cfg* cfg, fobf_server** out) {
  if (!cfg || !out) return fail(FOBF_EINVAL, "fobf_serve_create: NULL argument");
  if (cfg->hbm_budget_bytes == 0 || cfg->max_inflight < 1 || cfg->max_batch < 1 || cfg->R < 1 ||
      !(cfg->eps > 0.0))
    return fail(FOBF_EINVAL, "fobf_serve_create: invalid configuration");
  fobf_server* s = new fobf_server();
  s->cfg = *cfg;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fail(FOBF_EHIP, "fobf_serve_create: no HIP device");
  }
  for (int i = 0; i < kLanes; ++i) {
    if (hipStreamCreateWithFlags(&s->lanes[i], hipStreamNonBlocking) != hipSuccess) {
      for (int j = 0; j < i; ++j) hipStreamDestroy(s->lanes[j]);
      delete s;
      return fail(FOBF_EHIP, "fobf_serve_create: stream creation failed");
    }
  }
  if (hipMalloc(&s->d_coef, sizeof(float) * kCoefSlots * FOBF_KMAX) != hipSuccess) {
    for (int i = 0; i < kLanes; ++i) hipStreamDestroy(s->lanes[i]);
    delete s;
    return fail(FOBF_ENOMEM, "fobf_serve_create: coefficient table allocation failed");
  }
  // a private pool for request buffers: freed stream-ordered memory stays
  // resident between batches up to the budget, and beyond it is released;
  // the process's default pool is not touched
  {
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = s->device;
    if (hipMemPoolCreate(&s->pool, &props) == hipSuccess) {
      uint64_t thr = cfg->hbm_budget_bytes;
      hipMemPoolSetAttribute(s->pool, hipMemPoolAttrReleaseThreshold, &thr);
    } else {
      (void)hipGetLastError();
      s->pool = nullptr;
    }
  }
  s->worker = std::thread(worker_main, s);
  for (auto& f : s->fitters) f = std::thread(fitter_main, s);
  *out = s;
  return FOBF_OK;
}

extern "C" fobf_status fobf_serve_submit(fobf_server* s, const fobf_request* req,
                                         uint64_t* ticket) {
  if (!s || !req || !ticket) return fail(FOBF_EINVAL, "fobf_serve_submit: NULL argument");
  if (!req->h_in || !req->h_out || req->H < 1 || req->W < 1)
    return fail(FOBF_EINVAL, "fobf_serve_submit: bad image");
  if ((req->ld_in != 0 && req->ld_in < req->W) || (req->ld_out != 0 && req->ld_out < req->W))
    return fail(FOBF_EINVAL, "fobf_serve_submit: leading dimension below W");
  const int r = spatial_radius(req->theta);
  if (r < 1 || r > FOBF_RMAX) return fail(FOBF_EINVAL, "fobf_serve_submit: bad theta");
  if (!(req->sigma > 0.0) || !std::isfinite(req->sigma))
    return fail(FOBF_EINVAL, "fobf_serve_submit: bad sigma");
  if (req->K < 1 || req->K > FOBF_KMAX || req->K > s->cfg.R + 1)
    return fail(FOBF_EINVAL, "fobf_serve_submit: bad K");
  if (req->prec < FOBF_FP32 || req->prec > FOBF_FP16X2_STAGE)
    return fail(FOBF_EINVAL, "fobf_serve_submit: bad precision");
  if (!(req->deadline_s >= 0.0) || !std::isfinite(req->deadline_s))
    return fail(FOBF_EINVAL, "fobf_serve_submit: bad deadline");
  const size_t bytes = request_bytes(req->H, req->W, req->theta, req->prec);
  if (bytes > s->cfg.hbm_budget_bytes)
    return fail(FOBF_ENOMEM, "fobf_serve_submit: request larger than the HBM budget");
  Req* q = new Req();
  q->r = *req;
  if (q->r.ld_in == 0) q->r.ld_in = q->r.W;
  if (q->r.ld_out == 0) q->r.ld_out = q->r.W;
  q->bytes = bytes;
  uint64_t sb;
  std::memcpy(&sb, &req->sigma, sizeof(sb));
  q->key = CoefKey(s->cfg.R, sb, req->K);
  q->res.status = FOBF_EBUSY;
  q->res.t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete q;
      return fail(FOBF_ECANCELED, "fobf_serve_submit: server is stopping");
    }
    q->ticket = s->next_ticket++;
    s->stats.submitted += 1;
    if (s->coef.find(q->key) == s->coef.end()) {
      fobf_server::Coef e{};
      e.state = fobf_server::kFitting;
      s->coef.emplace(q->key, e);
      s->fit_queue.push_back(q->key);
      s->cv_fit.notify_one();
    }
    s->reqs[q->ticket] = q;
    s->pending.push_back(q);
    *ticket = q->ticket;
  }
  s->cv_work.notify_all();
  return FOBF_OK;
}

extern "C" fobf_status fobf_serve_poll(fobf_server* s, uint64_t ticket, int wait,
                                       fobf_result* res) {
  if (!s) return fail(FOBF_EINVAL, "fobf_serve_poll: NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(FOBF_EINVAL, "fobf_serve_poll: unknown ticket");
  Req* q = it->second;
  if (!q->done && wait) s->cv_done.wait(lk, [&]() { return q->done; });
  if (res) *res = q->res;
  if (!q->done) return FOBF_EBUSY;
  const fobf_status st = q->res.status;
  s->reqs.erase(it);
  delete q;
  if (st != FOBF_OK) set_error("fobf_serve_poll: request failed");
  return st;
}

extern "C" fobf_status fobf_serve_cancel(fobf_server* s, uint64_t ticket) {
  if (!s) return fail(FOBF_EINVAL, "fobf_serve_cancel: NULL server");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end() || it->second->done)
      return fail(FOBF_EINVAL, "fobf_serve_cancel: unknown or completed ticket");
    Req* q = it->second;
    auto pos = std::find(s->pending.begin(), s->pending.end(), q);
    if (pos == s->pending.end()) return FOBF_EBUSY;   // on the device: completes normally
    s->pending.erase(pos);
    q->res.status = FOBF_ECANCELED;
    q->res.t_done = now_s();
    q->done = true;
    s->stats.completed += 1;
    s->stats.failed += 1;
  }
  s->cv_done.notify_all();
  s->cv_work.notify_all();   // the queue head may have changed
  return FOBF_OK;
}

extern "C" fobf_status fobf_serve_inject_fault(fobf_server* s, int count) {
  if (!s || count < 0) return fail(FOBF_EINVAL, "fobf_serve_inject_fault: bad argument");
  std::lock_guard<std::mutex> lk(s->mu);
  s->inject = count;
  return FOBF_OK;
}

extern "C" fobf_status fobf_serve_get_stats(fobf_server* s, fobf_serve_stats* out) {
  if (!s || !out) return fail(FOBF_EINVAL, "fobf_serve_get_stats: NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  return FOBF_OK;
}

extern "C" fobf_status fobf_serve_destroy(fobf_server* s) {
  if (!s) return fail(FOBF_EINVAL, "fobf_serve_destroy: NULL server");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  s->cv_fit.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& f : s->fitters)
    if (f.joinable()) f.join();
  for (int i = 0; i < kLanes; ++i) {
    hipStreamSynchronize(s->lanes[i]);
    hipStreamDestroy(s->lanes[i]);
  }
  hipFree(s->d_coef);
  for (auto& kv : s->coef)
    if (kv.second.uploaded) hipEventDestroy(kv.second.uploaded);
  if (s->pool) hipMemPoolDestroy(s->pool);
  for (auto& kv : s->reqs) delete kv.second;
  delete s;
  return FOBF_OK;
}
