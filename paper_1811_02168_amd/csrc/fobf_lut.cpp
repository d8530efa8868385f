// Offline table of optimal (K*, T*) over a (sigma, eps) grid, read at run
// time by bilinear interpolation in (sigma, log(1/eps)) followed by one
// least-squares solve at the interpolated (K, T) (Sec. II, the paragraph
// after Algorithm 1, and Fig. 2).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fobf_internal.h"

namespace fobf {
fobf_status fit_at_period(int R, double sigma, int K, int T, double eps, fobf_coef* out);
}

using namespace fobf;

struct fobf_lut {
  int R = 0, Tmax = 0;
  std::vector<double> sigma, eps;      // grid: sigma increasing, eps decreasing
  std::vector<int> K, T;               // [i_sigma * n_eps + i_eps]
};

namespace {

bool valid_grid(const double* sigma, int ns, const double* eps, int ne) {
  if (ns < 1 || ne < 1 || !sigma || !eps) return false;
  for (int i = 0; i < ns; ++i)
    if (!(sigma[i] > 0.0) || !std::isfinite(sigma[i]) || (i && !(sigma[i] > sigma[i - 1])))
      return false;
  for (int j = 0; j < ne; ++j)
    if (!(eps[j] > 0.0) || !std::isfinite(eps[j]) || (j && !(eps[j] < eps[j - 1]))) return false;
  return true;
}

// Cell and weight of x in an increasing grid g[0..n-1]: x = (1-w) g[i] +
// w g[i+1] (i = 0, w = 0 for a one-point axis).  False outside the grid.
bool locate(const std::vector<double>& g, double x, int* i, double* w) {
  const int n = static_cast<int>(g.size());
  if (n == 1) {
    *i = 0;
    *w = 0.0;
    return x == g[0];
  }
  if (!(x >= g[0] && x <= g[n - 1])) return false;
  int k = static_cast<int>(std::upper_bound(g.begin(), g.end(), x) - g.begin()) - 1;
  k = std::min(std::max(k, 0), n - 2);
  *i = k;
  *w = (x - g[k]) / (g[k + 1] - g[k]);
  return true;
}

}  // namespace

extern "C" fobf_status fobf_lut_create(int R, const double* sigmas, int n_sigma,
                                       const double* eps, int n_eps, int Tmax,
                                       fobf_lut** out) {
  if (!out) return fail(FOBF_EINVAL, "fobf_lut_create: out is NULL");
  *out = nullptr;
  if (R < 1) return fail(FOBF_EINVAL, "fobf_lut_create: R must be >= 1");
  if (!valid_grid(sigmas, n_sigma, eps, n_eps))
    return fail(FOBF_EINVAL,
                "fobf_lut_create: need sigmas > 0 increasing and eps > 0 decreasing");
  if (Tmax <= 0) Tmax = 4 * R;
  fobf_lut* t = new fobf_lut();
  t->R = R;
  t->Tmax = Tmax;
  t->sigma.assign(sigmas, sigmas + n_sigma);
  t->eps.assign(eps, eps + n_eps);
  for (int i = 0; i < n_sigma; ++i)
    for (int j = 0; j < n_eps; ++j) {
      fobf_coef c;
      const fobf_status st = fobf_fit(R, sigmas[i], 0, eps[j], Tmax, &c);
      if (st != FOBF_OK) {
        delete t;
        return fail(FOBF_EINVAL, "fobf_lut_create: Algorithm 1 found no order for sigma " +
                                     std::to_string(sigmas[i]) + ", eps " +
                                     std::to_string(eps[j]));
      }
      t->K.push_back(c.K);
      t->T.push_back(c.T);
    }
  *out = t;
  return FOBF_OK;
}

extern "C" fobf_status fobf_lut_get(const fobf_lut* t, int i_sigma, int i_eps, int* K, int* T) {
  if (!t || !K || !T) return fail(FOBF_EINVAL, "fobf_lut_get: NULL argument");
  const int ns = static_cast<int>(t->sigma.size()), ne = static_cast<int>(t->eps.size());
  if (i_sigma < 0 || i_sigma >= ns || i_eps < 0 || i_eps >= ne)
    return fail(FOBF_EINVAL, "fobf_lut_get: index out of range");
  *K = t->K[i_sigma * ne + i_eps];
  *T = t->T[i_sigma * ne + i_eps];
  return FOBF_OK;
}

extern "C" fobf_status fobf_lut_fit(const fobf_lut* t, double sigma, double eps,
                                    fobf_coef* out) {
  if (!t || !out) return fail(FOBF_EINVAL, "fobf_lut_fit: NULL argument");
  if (!(sigma > 0.0) || !(eps > 0.0) || !std::isfinite(sigma) || !std::isfinite(eps))
    return fail(FOBF_EINVAL, "fobf_lut_fit: sigma and eps must be positive and finite");
  // the eps axis is interpolated in L = log(1/eps), increasing along it
  std::vector<double> L(t->eps.size());
  for (size_t j = 0; j < L.size(); ++j) L[j] = -std::log(t->eps[j]);
  int i, j;
  double ws, wl;
  if (!locate(t->sigma, sigma, &i, &ws) || !locate(L, -std::log(eps), &j, &wl))
    return fail(FOBF_EINVAL, "fobf_lut_fit: (sigma, eps) outside the table");
  const int ne = static_cast<int>(t->eps.size());
  const int i1 = t->sigma.size() > 1 ? i + 1 : i, j1 = ne > 1 ? j + 1 : j;
  auto bil = [&](const std::vector<int>& v) {
    return (1 - ws) * ((1 - wl) * v[i * ne + j] + wl * v[i * ne + j1]) +
           ws * ((1 - wl) * v[i1 * ne + j] + wl * v[i1 * ne + j1]);
  };
  // order rounded up (never fewer terms than the interpolation suggests),
  // period to the nearest integer, at least K - 1 (full rank)
  const int K = std::min(FOBF_KMAX, static_cast<int>(std::ceil(bil(t->K) - 1e-9)));
  const int T = std::max(std::max(1, K - 1), static_cast<int>(std::lround(bil(t->T))));
  const fobf_status st = fit_at_period(t->R, sigma, K, T, eps, out);
  out->Tmax = t->Tmax;
  return st;
}

extern "C" fobf_status fobf_lut_save(const fobf_lut* t, const char* path) {
  if (!t || !path) return fail(FOBF_EINVAL, "fobf_lut_save: NULL argument");
  FILE* fp = std::fopen(path, "w");
  if (!fp) return fail(FOBF_EINVAL, std::string("fobf_lut_save: cannot open ") + path);
  std::fprintf(fp, "# fobf (K*, T*) table v1: R Tmax n_sigma n_eps; sigmas; eps; K T rows\n");
  std::fprintf(fp, "%d %d %zu %zu\n", t->R, t->Tmax, t->sigma.size(), t->eps.size());
  for (double v : t->sigma) std::fprintf(fp, "%.17g ", v);
  std::fprintf(fp, "\n");
  for (double v : t->eps) std::fprintf(fp, "%.17g ", v);
  std::fprintf(fp, "\n");
  for (size_t n = 0; n < t->K.size(); ++n) std::fprintf(fp, "%d %d\n", t->K[n], t->T[n]);
  const bool ok = std::fclose(fp) == 0;
  return ok ? FOBF_OK : fail(FOBF_EINVAL, "fobf_lut_save: write failed");
}

extern "C" fobf_status fobf_lut_load(const char* path, fobf_lut** out) {
  if (!path || !out) return fail(FOBF_EINVAL, "fobf_lut_load: NULL argument");
  *out = nullptr;
  FILE* fp = std::fopen(path, "r");
  if (!fp) return fail(FOBF_EINVAL, std::string("fobf_lut_load: cannot open ") + path);
  fobf_lut* t = new fobf_lut();
  char line[512];
  bool ok = std::fgets(line, sizeof(line), fp) && line[0] == '#';
  int ns = 0, ne = 0;
  ok = ok && std::fscanf(fp, "%d %d %d %d", &t->R, &t->Tmax, &ns, &ne) == 4 && t->R >= 1 &&
       t->Tmax >= 1 && ns >= 1 && ne >= 1 && ns <= 100000 && ne <= 100000;
  if (ok) {
    t->sigma.resize(ns);
    t->eps.resize(ne);
    for (int i = 0; ok && i < ns; ++i) ok = std::fscanf(fp, "%lf", &t->sigma[i]) == 1;
    for (int j = 0; ok && j < ne; ++j) ok = std::fscanf(fp, "%lf", &t->eps[j]) == 1;
    ok = ok && valid_grid(t->sigma.data(), ns, t->eps.data(), ne);
    for (int n = 0; ok && n < ns * ne; ++n) {
      int K, T;
      ok = std::fscanf(fp, "%d %d", &K, &T) == 2 && K >= 1 && K <= FOBF_KMAX &&
           T >= std::max(1, K - 1);
      t->K.push_back(K);
      t->T.push_back(T);
    }
  }
  std::fclose(fp);
  if (!ok) {
    delete t;
    return fail(FOBF_EINVAL, std::string("fobf_lut_load: malformed table ") + path);
  }
  *out = t;
  return FOBF_OK;
}

extern "C" void fobf_lut_destroy(fobf_lut* t) { delete t; }
