// Post-processing of a gap-ratio sweep (section "Effect of Gap Ratio"): the cubic
// least-squares fit of CoPFI over delta with its R^2 and mean square error.  A few
// hundred host values at most, so host code: Householder QR of the n x 4 matrix
// [x^3 x^2 x 1], then back substitution.
#include <cmath>
#include <vector>

#include "mfp_internal.h"

using namespace mfp;

extern "C" int mfp_cubic_fit(const double* x_h, const double* y_h, int32_t n, double* coef_h,
                             double* r2_h, double* mse_h) {
  clear_error();
  if (!x_h || !y_h || !coef_h) {
    set_error("NULL argument");
    return MFP_E_ARG;
  }
  if (n < 4) {
    set_error("a cubic fit needs at least 4 points (got %d)", n);
    return MFP_E_ARG;
  }
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(x_h[i]) || !std::isfinite(y_h[i])) {
      set_error("non-finite value at %d", i);
      return MFP_E_ARG;
    }
  // A (column-major, n x 4) and the right-hand side
  std::vector<double> A(4 * (size_t)n), b(y_h, y_h + n);
  for (int i = 0; i < n; ++i) {
    const double x = x_h[i];
    A[i] = x * x * x;
    A[n + i] = x * x;
    A[2 * (size_t)n + i] = x;
    A[3 * (size_t)n + i] = 1.0;
  }
  double R[4][4] = {};
  for (int k = 0; k < 4; ++k) {
    double* a = &A[(size_t)k * n];
    double nrm = 0.0;
    for (int i = k; i < n; ++i) nrm += a[i] * a[i];
    nrm = std::sqrt(nrm);
    double scale = 0.0;
    for (int c = 0; c < 4; ++c) {
      const double* ac = &A[(size_t)c * n];
      for (int i = 0; i < n; ++i) scale = std::fmax(scale, std::fabs(ac[i]));
    }
    if (!(nrm > 1e-13 * scale * std::sqrt((double)n))) {
      set_error("x has fewer than 4 distinct values (rank-deficient fit)");
      return MFP_E_ARG;
    }
    // Householder vector v = a_k.. + sign(a_kk) |a| e_k, stored in place
    const double alpha = a[k] >= 0.0 ? -nrm : nrm;
    a[k] -= alpha;
    double vv = 0.0;
    for (int i = k; i < n; ++i) vv += a[i] * a[i];
    // apply H = I - 2 v v^T / (v^T v) to the later columns and to b
    for (int c = k + 1; c < 4; ++c) {
      double* ac = &A[(size_t)c * n];
      double d = 0.0;
      for (int i = k; i < n; ++i) d += a[i] * ac[i];
      const double f = 2.0 * d / vv;
      for (int i = k; i < n; ++i) ac[i] -= f * a[i];
    }
    double d = 0.0;
    for (int i = k; i < n; ++i) d += a[i] * b[i];
    const double f = 2.0 * d / vv;
    for (int i = k; i < n; ++i) b[i] -= f * a[i];
    R[k][k] = alpha;
    for (int c = k + 1; c < 4; ++c) R[k][c] = A[(size_t)c * n + k];
  }
  double c[4];
  for (int k = 3; k >= 0; --k) {
    double s = b[k];
    for (int m = k + 1; m < 4; ++m) s -= R[k][m] * c[m];
    c[k] = s / R[k][k];
  }
  double mean = 0.0;
  for (int i = 0; i < n; ++i) mean += y_h[i];
  mean /= n;
  double ss_res = 0.0, ss_tot = 0.0;
  for (int i = 0; i < n; ++i) {
    const double x = x_h[i];
    const double r = y_h[i] - (((c[0] * x + c[1]) * x + c[2]) * x + c[3]);
    ss_res += r * r;
    ss_tot += (y_h[i] - mean) * (y_h[i] - mean);
  }
  for (int k = 0; k < 4; ++k) coef_h[k] = c[k];
  if (r2_h) *r2_h = ss_tot > 0.0 ? 1.0 - ss_res / ss_tot : 1.0;
  if (mse_h) *mse_h = ss_res / n;
  return MFP_OK;
}
