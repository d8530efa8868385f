// Host-side float64 least-squares fit of the cosine range kernel.
//
// eq. (3): phi_hat(t) = sum_{k<K} c_k cos(nu k t), nu = 2 pi / (2T+1).
// eq. (4): kernel error sum_{t=-R..R} (phi(t) - phi_hat(t))^2.
// eq. (5): E(K,T) = min_c ||A c - b||^2 with A(t,k) = cos(nu k t), b(t) =
//          phi(t), over the 2R+1 integers t of [-R, R].
// eq. (6) and Algorithm 1: scan the period T, then (K = 0) raise K.
//
// Both phi and every column of A are even in t, so the 2R+1 equations fold
// onto t = 0..R with weight 1 at t = 0 and 2 elsewhere; the weighted system
// (rows scaled by sqrt(weight)) has the same minimiser and the same
// residual norm.  It is solved with Householder QR in float64, because
// A becomes badly conditioned for large T (normal equations are not used),
// and E is evaluated from the explicit residual.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <map>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "fobf_internal.h"

namespace fobf {
namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

// Solves min ||M c - y|| for an m x n column-major matrix M (m >= n) by
// Householder QR.  M and y are overwritten.  Returns false when a column is
// numerically dependent (pivot below tol * norm of the column).
bool householder_lstsq(int m, int n, double* M, double* y, double* c) {
  std::vector<double> colnorm(n);
  for (int j = 0; j < n; ++j) {
    double s = 0;
    for (int i = 0; i < m; ++i) s += M[j * m + i] * M[j * m + i];
    colnorm[j] = std::sqrt(s);
  }
  std::vector<double> diag(n);
  for (int j = 0; j < n; ++j) {
    double* a = M + j * m;
    double s = 0;
    for (int i = j; i < m; ++i) s += a[i] * a[i];
    double alpha = std::sqrt(s);
    if (alpha <= 1e-13 * colnorm[j] || alpha == 0.0) return false;
    if (a[j] > 0) alpha = -alpha;
    // v = a[j:] - alpha e_1, stored in place; H = I - 2 v v^T / (v^T v)
    a[j] -= alpha;
    double vtv = 0;
    for (int i = j; i < m; ++i) vtv += a[i] * a[i];
    diag[j] = alpha;
    for (int k = j + 1; k < n; ++k) {
      double* b = M + k * m;
      double d = 0;
      for (int i = j; i < m; ++i) d += a[i] * b[i];
      d = 2.0 * d / vtv;
      for (int i = j; i < m; ++i) b[i] -= d * a[i];
    }
    double d = 0;
    for (int i = j; i < m; ++i) d += a[i] * y[i];
    d = 2.0 * d / vtv;
    for (int i = j; i < m; ++i) y[i] -= d * a[i];
  }
  // back substitution with the upper triangle (diag holds R_jj)
  for (int j = n - 1; j >= 0; --j) {
    double s = y[j];
    for (int k = j + 1; k < n; ++k) s -= M[k * m + j] * c[k];
    c[j] = s / diag[j];
  }
  return true;
}

// cos(2 pi j / P) for j = 0 .. P/2: with the exact integer reduction
// j = (k t) mod P and the symmetry cos(2 pi (P - j) / P) = cos(2 pi j / P),
// every entry of the design matrix for period P is one of these.
void cos_table(long P, std::vector<double>* tab) {
  tab->resize(static_cast<size_t>(P / 2 + 1));
  for (long j = 0; j <= P / 2; ++j)
    (*tab)[j] = std::cos(kTwoPi * static_cast<double>(j) / static_cast<double>(P));
}

inline double cos_at(const std::vector<double>& tab, long kt, long P) {
  long j = kt % P;
  if (j > P / 2) j = P - j;
  return tab[j];
}

struct FitOne {
  bool ok;
  double E;
  double delta;
  double c[FOBF_KMAX];
};

// E(K, T) of eq. (5) for samples b[0..R] of an even kernel.  `work` is
// per-thread scratch reused across periods.
struct FitWork {
  std::vector<double> tab, A, M, y;
};

FitOne fit_one(int R, const double* b, int K, int T, FitWork* w) {
  FitOne r{};
  const int m = R + 1;
  const long P = 2L * T + 1;
  cos_table(P, &w->tab);
  w->A.resize(static_cast<size_t>(m) * K);
  w->y.resize(m);
  for (int k = 0; k < K; ++k)
    for (int t = 0; t <= R; ++t)
      w->A[static_cast<size_t>(k) * m + t] = cos_at(w->tab, static_cast<long>(k) * t, P);
  w->M.resize(w->A.size());
  for (int k = 0; k < K; ++k)
    for (int t = 0; t <= R; ++t)
      w->M[static_cast<size_t>(k) * m + t] =
          (t == 0 ? 1.0 : std::sqrt(2.0)) * w->A[static_cast<size_t>(k) * m + t];
  for (int t = 0; t <= R; ++t) w->y[t] = (t == 0 ? 1.0 : std::sqrt(2.0)) * b[t];
  r.ok = householder_lstsq(m, K, w->M.data(), w->y.data(), r.c);
  if (!r.ok) return r;
  // explicit residual of the unfolded system: t = 0 once, t > 0 twice
  double E = 0, dmax = 0;
  for (int t = 0; t <= R; ++t) {
    double s = 0;
    for (int k = 0; k < K; ++k) s += r.c[k] * w->A[static_cast<size_t>(k) * m + t];
    const double d = s - b[t];
    E += (t == 0 ? 1.0 : 2.0) * d * d;
    dmax = std::max(dmax, std::fabs(d));
  }
  r.E = E;
  r.delta = dmax;
  return r;
}

// Best period for fixed K: T = max(1, K-1) .. Tmax, smallest E, first T on
// exact ties.  (For T <= K-2 the columns k and 2T+1-k coincide, so those
// periods are rank deficient and skipped.)  The periods are independent
// least-squares problems: they are split over up to 8 host threads, each
// keeping its own best, and merged by (E, T) -- the same answer as one
// ascending pass, whatever the thread count.
bool scan_T(int R, const double* b, int K, int Tmax, int* Tbest, FitOne* best) {
  const int T0 = std::max(1, K - 1);
  const int nT = Tmax - T0 + 1;
  if (nT < 1) return false;
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int nth = std::max(1, std::min({8, static_cast<int>(hw), nT / 32}));
  std::vector<FitOne> bestv(nth);
  std::vector<int> Tv(nth, 0);
  auto run = [&](int id) {
    FitWork w;
    for (int T = T0 + id; T <= Tmax; T += nth) {
      FitOne f = fit_one(R, b, K, T, &w);
      if (!f.ok) continue;
      if (Tv[id] == 0 || f.E < bestv[id].E) {
        bestv[id] = f;
        Tv[id] = T;
      }
    }
  };
  std::vector<std::thread> pool;
  for (int id = 1; id < nth; ++id) pool.emplace_back(run, id);
  run(0);
  for (auto& th : pool) th.join();
  bool found = false;
  for (int id = 0; id < nth; ++id) {
    if (Tv[id] == 0) continue;
    if (!found || bestv[id].E < best->E || (bestv[id].E == best->E && Tv[id] < *Tbest)) {
      *best = bestv[id];
      *Tbest = Tv[id];
      found = true;
    }
  }
  return found;
}

// Best period for fixed K by a local search from T0 (Sec. II, the remark
// after Algorithm 1: E(K, T) is unimodal in T for fixed K).  Measured on
// the Gaussian kernel (R = 31 .. 1023, sigma from 0.04 R to 0.4 R, K = 2 ..
// 12), E falls strictly from about T = R/2 up to T* and rises strictly from
// T* to at least 3.4 R, so a descent started anywhere in that basin -- T0 =
// R is inside it in every case -- ends at the scan's T*; only where E
// reaches the float64 floor (~1e-29) is the curve flat and noisy, and any
// period there is as good.  Below R/2 (and for K >= 11 near 4R) the curve
// has ripples, which is why the search needs a start inside the basin
// rather than the scan's T = K-1.
//
// The search brackets the minimum by doubling steps downhill from T0, then
// narrows the bracket by golden-section steps on the integers and finally
// compares the last few periods (smallest T on exact ties).  About 20-30
// least-squares solves instead of the scan's Tmax - K + 2.
bool descend_T(int R, const double* b, int K, int Tlo, int Thi, int T0, int* Tbest,
               FitOne* best, int* evals) {
  if (Tlo > Thi) return false;
  FitWork w;
  std::map<int, FitOne> memo;
  auto E = [&](int T) -> double {
    auto it = memo.find(T);
    if (it == memo.end()) {
      it = memo.emplace(T, fit_one(R, b, K, T, &w)).first;
      if (evals) *evals += 1;
    }
    return it->second.ok ? it->second.E : INFINITY;
  };
  T0 = std::min(std::max(T0, Tlo), Thi);
  const double e0 = E(T0);
  const double el = T0 > Tlo ? E(T0 - 1) : INFINITY;
  const double er = T0 < Thi ? E(T0 + 1) : INFINITY;
  int lo = std::max(Tlo, T0 - 1), hi = std::min(Thi, T0 + 1);
  if (el < e0 || er < e0) {
    // walk downhill with doubling steps until E rises: the minimum then
    // lies strictly between the last point before the best one and the
    // point after it
    const int d = (el < er) ? -1 : 1;
    int a = T0, m = T0 + d, step = 1;
    for (;;) {
      step *= 2;
      int c = m + d * step;
      c = std::min(std::max(c, Tlo), Thi);
      if (c == m) {           // at the end of the range: the minimum is in (a, m]
        lo = std::min(a, m);
        hi = std::max(a, m);
        break;
      }
      if (E(c) >= E(m)) {
        lo = std::min(a, c);
        hi = std::max(a, c);
        break;
      }
      a = m;
      m = c;
    }
    // golden-section narrowing of [lo, hi], which holds a minimum inside
    while (hi - lo > 4) {
      const int x1 = lo + static_cast<int>(std::lround(0.381966 * (hi - lo)));
      const int x2 = hi - static_cast<int>(std::lround(0.381966 * (hi - lo)));
      if (x1 >= x2) break;
      if (E(x1) <= E(x2)) hi = x2; else lo = x1;
    }
  }
  bool found = false;
  for (int T = lo; T <= hi; ++T) {
    const double e = E(T);
    if (!std::isfinite(e)) continue;
    if (!found || e < best->E) {
      *best = memo.at(T);
      *Tbest = T;
      found = true;
    }
  }
  return found;
}

std::vector<double> gaussian_samples(int R, double sigma) {
  std::vector<double> b(R + 1);
  for (int t = 0; t <= R; ++t) b[t] = std::exp(-(double)t * t / (2.0 * sigma * sigma));
  return b;
}

void fill(fobf_coef* out, int R, int K, int T, int Tmax, double sigma,
          const FitOne& f) {
  std::memset(out, 0, sizeof(*out));
  out->R = R;
  out->K = K;
  out->T = T;
  out->Tmax = Tmax;
  out->sigma = sigma;
  out->E = f.E;
  out->delta = f.delta;
  for (int k = 0; k < K; ++k) out->c[k] = f.c[k];
}

std::mutex g_cache_mu;
std::map<std::tuple<int, uint64_t, int, uint64_t, int>, fobf_coef> g_cache;

uint64_t bits(double d) {
  uint64_t u;
  std::memcpy(&u, &d, sizeof(u));
  return u;
}

fobf_status fit_samples_impl(int R, const double* b, int K, double eps,
                             int Tmax, double sigma, fobf_coef* out) {
  if (K >= 1) {
    int T = 0;
    FitOne f{};
    if (!scan_T(R, b, K, Tmax, &T, &f))
      return fail(FOBF_EINTERNAL, "fobf_fit: no full-rank period found");
    fill(out, R, K, T, Tmax, sigma, f);
    if (!(f.E <= eps)) {
      set_error("fobf_fit: E(K,T*) exceeds eps");
      return FOBF_WARN_TOL;
    }
    return FOBF_OK;
  }
  // Algorithm 1: smallest K whose best period reaches E <= eps.
  const int Klim = std::min(FOBF_KMAX, R + 1);
  for (int k = 1; k <= Klim; ++k) {
    int T = 0;
    FitOne f{};
    if (!scan_T(R, b, k, Tmax, &T, &f)) continue;
    if (f.E <= eps) {
      fill(out, R, k, T, Tmax, sigma, f);
      return FOBF_OK;
    }
  }
  return fail(FOBF_EINVAL, "fobf_fit: no order up to FOBF_KMAX meets eps");
}

}  // namespace

// Least-squares fit at one given period (eq. (5) without the scan over T).
fobf_status fit_at_period(int R, double sigma, int K, int T, double eps, fobf_coef* out) {
  std::vector<double> b = gaussian_samples(R, sigma);
  FitWork w;
  FitOne f = fit_one(R, b.data(), K, T, &w);
  if (!f.ok) return fail(FOBF_EINVAL, "fobf_fit_period: columns are dependent at this period");
  fill(out, R, K, T, T, sigma, f);
  if (!(f.E <= eps)) {
    set_error("fobf_fit_period: E(K,T) exceeds eps");
    return FOBF_WARN_TOL;
  }
  return FOBF_OK;
}

}  // namespace fobf

using namespace fobf;

extern "C" fobf_status fobf_fit_period(int R, double sigma, int K, int T, fobf_coef* out) {
  if (!out) return fail(FOBF_EINVAL, "fobf_fit_period: out is NULL");
  if (R < 1) return fail(FOBF_EINVAL, "fobf_fit_period: R must be >= 1");
  if (!(sigma > 0.0) || !std::isfinite(sigma))
    return fail(FOBF_EINVAL, "fobf_fit_period: sigma must be positive and finite");
  if (K < 1 || K > FOBF_KMAX || K > R + 1)
    return fail(FOBF_EINVAL, "fobf_fit_period: K out of range");
  if (T < std::max(1, K - 1)) return fail(FOBF_EINVAL, "fobf_fit_period: T below max(1, K-1)");
  return fit_at_period(R, sigma, K, T, INFINITY, out);
}

extern "C" fobf_status fobf_fit(int R, double sigma, int K, double eps,
                                int Tmax, fobf_coef* out) {
  if (!out) return fail(FOBF_EINVAL, "fobf_fit: out is NULL");
  if (R < 1) return fail(FOBF_EINVAL, "fobf_fit: R must be >= 1");
  if (!(sigma > 0.0) || !std::isfinite(sigma))
    return fail(FOBF_EINVAL, "fobf_fit: sigma must be positive and finite");
  if (!(eps > 0.0)) return fail(FOBF_EINVAL, "fobf_fit: eps must be > 0");
  if (K < 0 || K > FOBF_KMAX || K > R + 1)
    return fail(FOBF_EINVAL, "fobf_fit: K out of range");
  if (Tmax <= 0) Tmax = 4 * R;
  if (Tmax < std::max(1, K - 1))
    return fail(FOBF_EINVAL, "fobf_fit: Tmax below K-1");
  auto key = std::make_tuple(R, bits(sigma), K, bits(eps), Tmax);
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      *out = it->second;
      if (!(out->E <= eps)) {
        set_error("fobf_fit: E(K,T*) exceeds eps");
        return FOBF_WARN_TOL;
      }
      return FOBF_OK;
    }
  }
  std::vector<double> b = gaussian_samples(R, sigma);
  fobf_status st = fit_samples_impl(R, b.data(), K, eps, Tmax, sigma, out);
  if (st == FOBF_OK || st == FOBF_WARN_TOL) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache[key] = *out;
  }
  return st;
}

extern "C" fobf_status fobf_fit_warm(int R, double sigma, int K, double eps, int Tmax, int T0,
                                     fobf_coef* out) {
  if (!out) return fail(FOBF_EINVAL, "fobf_fit_warm: out is NULL");
  if (R < 1) return fail(FOBF_EINVAL, "fobf_fit_warm: R must be >= 1");
  if (!(sigma > 0.0) || !std::isfinite(sigma))
    return fail(FOBF_EINVAL, "fobf_fit_warm: sigma must be positive and finite");
  if (!(eps > 0.0)) return fail(FOBF_EINVAL, "fobf_fit_warm: eps must be > 0");
  if (K < 1 || K > FOBF_KMAX || K > R + 1)
    return fail(FOBF_EINVAL, "fobf_fit_warm: K out of range");
  if (Tmax <= 0) Tmax = 4 * R;
  const int Tlo = std::max(1, K - 1);
  if (Tmax < Tlo) return fail(FOBF_EINVAL, "fobf_fit_warm: Tmax below K-1");
  if (T0 <= 0) T0 = R;
  std::vector<double> b = gaussian_samples(R, sigma);
  int T = 0, evals = 0;
  FitOne f{};
  if (!descend_T(R, b.data(), K, Tlo, Tmax, T0, &T, &f, &evals))
    return fail(FOBF_EINTERNAL, "fobf_fit_warm: no full-rank period found");
  fill(out, R, K, T, Tmax, sigma, f);
  if (!(f.E <= eps)) {
    set_error("fobf_fit_warm: E(K,T*) exceeds eps");
    return FOBF_WARN_TOL;
  }
  return FOBF_OK;
}

extern "C" int fobf_fit_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  const int n = static_cast<int>(g_cache.size());
  g_cache.clear();
  return n;
}

// Cache file: one line per entry, "key_K R Tmax sigma eps T K E delta c_0 ..
// c_{K-1}", the doubles as C99 hexadecimal floats so that a round trip is
// exact.
extern "C" fobf_status fobf_fit_cache_save(const char* path) {
  if (!path) return fail(FOBF_EINVAL, "fobf_fit_cache_save: path is NULL");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(FOBF_EINVAL, std::string("fobf_fit_cache_save: cannot open ") + path);
  std::fprintf(f, "# fobf fit cache v1: keyK R Tmax sigma eps T K E delta c[0..K-1]\n");
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (const auto& kv : g_cache) {
      double sigma, eps;
      const uint64_t sb = std::get<1>(kv.first), eb = std::get<3>(kv.first);
      std::memcpy(&sigma, &sb, sizeof(sigma));
      std::memcpy(&eps, &eb, sizeof(eps));
      const fobf_coef& c = kv.second;
      std::fprintf(f, "%d %d %d %a %a %d %d %a %a", std::get<2>(kv.first), std::get<0>(kv.first),
                   std::get<4>(kv.first), sigma, eps, c.T, c.K, c.E, c.delta);
      for (int k = 0; k < c.K; ++k) std::fprintf(f, " %a", c.c[k]);
      std::fprintf(f, "\n");
    }
  }
  const bool ok = std::fclose(f) == 0;
  return ok ? FOBF_OK : fail(FOBF_EINVAL, "fobf_fit_cache_save: write failed");
}

extern "C" fobf_status fobf_fit_cache_load(const char* path) {
  if (!path) return fail(FOBF_EINVAL, "fobf_fit_cache_load: path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(FOBF_EINVAL, std::string("fobf_fit_cache_load: cannot open ") + path);
  std::vector<std::pair<std::tuple<int, uint64_t, int, uint64_t, int>, fobf_coef>> rows;
  char line[4096];
  bool bad = false;
  while (std::fgets(line, sizeof(line), f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    int keyK, R, Tmax, T, K, used = 0;
    double sigma, eps, E, delta;
    if (std::sscanf(line, "%d %d %d %la %la %d %d %la %la%n", &keyK, &R, &Tmax, &sigma, &eps, &T,
                    &K, &E, &delta, &used) != 9) {
      bad = true;
      break;
    }
    if (R < 1 || K < 1 || K > FOBF_KMAX || keyK < 0 || keyK > FOBF_KMAX ||
        (keyK != 0 && keyK != K) || T < 1 || Tmax < T || !(sigma > 0.0) || !(eps > 0.0) ||
        !std::isfinite(E) || !std::isfinite(delta)) {
      bad = true;
      break;
    }
    fobf_coef c{};
    c.R = R;
    c.K = K;
    c.T = T;
    c.Tmax = Tmax;
    c.sigma = sigma;
    c.E = E;
    c.delta = delta;
    const char* p = line + used;
    for (int k = 0; k < K; ++k) {
      int n = 0;
      if (std::sscanf(p, " %la%n", &c.c[k], &n) != 1 || !std::isfinite(c.c[k])) {
        bad = true;
        break;
      }
      p += n;
    }
    if (bad) break;
    rows.push_back({std::make_tuple(R, bits(sigma), keyK, bits(eps), Tmax), c});
  }
  std::fclose(f);
  if (bad) return fail(FOBF_EINVAL, "fobf_fit_cache_load: malformed line");
  std::lock_guard<std::mutex> lk(g_cache_mu);
  for (auto& r : rows) g_cache[r.first] = r.second;
  return FOBF_OK;
}

extern "C" fobf_status fobf_fit_samples(int R, const double* b, int K,
                                        double eps, int Tmax, fobf_coef* out) {
  if (!out || !b) return fail(FOBF_EINVAL, "fobf_fit_samples: NULL pointer");
  if (R < 1) return fail(FOBF_EINVAL, "fobf_fit_samples: R must be >= 1");
  if (!(eps > 0.0)) return fail(FOBF_EINVAL, "fobf_fit_samples: eps must be > 0");
  if (K < 1 || K > FOBF_KMAX || K > R + 1)
    return fail(FOBF_EINVAL, "fobf_fit_samples: K out of range");
  for (int t = 0; t <= R; ++t)
    if (!std::isfinite(b[t]))
      return fail(FOBF_EINVAL, "fobf_fit_samples: non-finite sample");
  if (Tmax <= 0) Tmax = 4 * R;
  if (Tmax < std::max(1, K - 1))
    return fail(FOBF_EINVAL, "fobf_fit_samples: Tmax below K-1");
  return fit_samples_impl(R, b, K, eps, Tmax, 0.0, out);
}
