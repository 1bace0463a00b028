// Small dense host linear algebra for the offline gPC stage.
//  * householder_lstsq: least-squares fit of the gPC coefficients (eq. least square
//    problem) by Householder QR of the design matrix and back substitution.
#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <vector>

#include "common.h"

namespace kc {

// min |B X - D| with B [m][n] (m >= n), D [m][nrhs], both row-major (overwritten).
// Returns KC_OK or KC_ERANK.
int householder_lstsq(int m, int n, int nrhs, std::vector<double>& B, std::vector<double>& D,
                      std::vector<double>& X) {
  if (m < n) return KC_ERANK;
  std::vector<double> v(m);
  std::vector<double> rdiag(n);
  auto b = [&](int r, int c) -> double& { return B[(size_t)r * n + c]; };
  for (int k = 0; k < n; ++k) {
    double nrm = 0.0;
    for (int i = k; i < m; ++i) nrm = std::hypot(nrm, b(i, k));
    const double alpha = b(k, k) >= 0 ? -nrm : nrm;
    rdiag[k] = alpha;
    if (nrm == 0.0) continue;
    for (int i = k; i < m; ++i) v[i] = b(i, k);
    v[k] -= alpha;
    double vv = 0.0;
    for (int i = k; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double beta = 2.0 / vv;
    for (int c = k + 1; c < n; ++c) {
      double s = 0.0;
      for (int i = k; i < m; ++i) s += v[i] * b(i, c);
      s *= beta;
      for (int i = k; i < m; ++i) b(i, c) -= s * v[i];
    }
    for (int c = 0; c < nrhs; ++c) {
      double s = 0.0;
      for (int i = k; i < m; ++i) s += v[i] * D[(size_t)i * nrhs + c];
      s *= beta;
      for (int i = k; i < m; ++i) D[(size_t)i * nrhs + c] -= s * v[i];
    }
  }
  double rmax = 0.0;
  for (int k = 0; k < n; ++k) rmax = std::max(rmax, std::fabs(rdiag[k]));
  for (int k = 0; k < n; ++k)
    if (!(std::fabs(rdiag[k]) > 1e-12 * rmax)) return KC_ERANK;
  X.assign((size_t)n * nrhs, 0.0);
  for (int c = 0; c < nrhs; ++c) {
    for (int k = n - 1; k >= 0; --k) {
      double s = D[(size_t)k * nrhs + c];
      for (int j = k + 1; j < n; ++j) s -= b(k, j) * X[(size_t)j * nrhs + c];
      X[(size_t)k * nrhs + c] = s / rdiag[k];
    }
  }
  return KC_OK;
}

}  // namespace kc
