// Two-level estimator of a factorized observable (Section 3.1): level-1 means
// of the two factors, each over the updates of its own region, their product
// per level-0 field, and the level-0 mean with its standard error; the other
// pieces are binned per level-0 field.  Host arithmetic on the small arrays of
// per-update measurements (contraction outputs copied back).
#include <cmath>
#include <vector>

#include "../../include/ddml.h"

namespace {

// mean and standard error (n - 1 in the variance) of n values with stride s
void mean_err(const double* v, int n, size_t s, double* mean, double* err) {
  double m = 0;
  for (int i = 0; i < n; ++i) m += v[i * s];
  m /= n;
  double q = 0;
  for (int i = 0; i < n; ++i) q += (v[i * s] - m) * (v[i * s] - m);
  *mean = m;
  *err = n > 1 ? std::sqrt(q / (n - 1) / n) : 0.0;
}

}  // namespace

extern "C" int ddml_two_level_average(int n0, int n1, int nc, int ma, int mb, const double* a, const double* b,
                                      int k, const double* rest, double* est_f, double* err_f, double* est_r,
                                      double* err_r) {
  if (n0 < 1 || n1 < 1 || nc < 1 || ma < 1 || mb < 1 || k < 0 || !a || !b || !est_f || !err_f) return DDML_EINVAL;
  if (k > 0 && (!rest || !est_r || !err_r)) return DDML_EINVAL;
  const size_t na = (size_t)nc * ma, nb = (size_t)nc * mb, np = (size_t)ma * mb;
  std::vector<double> Ma(na), Mb(nb), P((size_t)n0 * np);
  for (int i = 0; i < n0; ++i) {
    // level-1 means of each region's factor for level-0 field i
    for (size_t e = 0; e < na; ++e) {
      double s = 0;
      for (int j = 0; j < n1; ++j) s += a[((size_t)i * n1 + j) * na + e];
      Ma[e] = s / n1;
    }
    for (size_t e = 0; e < nb; ++e) {
      double s = 0;
      for (int j = 0; j < n1; ++j) s += b[((size_t)i * n1 + j) * nb + e];
      Mb[e] = s / n1;
    }
    for (int x = 0; x < ma; ++x)
      for (int y = 0; y < mb; ++y) {
        double s = 0;
        for (int c = 0; c < nc; ++c) s += Ma[(size_t)c * ma + x] * Mb[(size_t)c * mb + y];
        P[(size_t)i * np + (size_t)x * mb + y] = s;
      }
  }
  for (size_t e = 0; e < np; ++e) mean_err(P.data() + e, n0, np, est_f + e, err_f + e);
  if (k > 0) {
    std::vector<double> bins((size_t)n0 * k);
    for (int i = 0; i < n0; ++i)
      for (int r = 0; r < k; ++r) {
        double s = 0;
        for (int j = 0; j < n1; ++j) s += rest[((size_t)i * n1 + j) * k + r];
        bins[(size_t)i * k + r] = s / n1;
      }
    for (int r = 0; r < k; ++r) mean_err(bins.data() + r, n0, k, est_r + r, err_r + r);
  }
  return DDML_OK;
}
