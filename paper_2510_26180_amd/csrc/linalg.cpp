// Small dense host linear algebra for the offline KL / gPC stages.
//  * sym_eig: eigen-decomposition of the n_t x n_t snapshot covariance (Section 2.1):
//    Householder reduction to tridiagonal form, then implicit QL sweeps with Wilkinson-
//    type shifts, both accumulating the orthogonal transformation.
//  * householder_lstsq: least-squares fit of the gPC coefficients (eq. least square
//    problem) by Householder QR of the design matrix and back substitution.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "common.h"

namespace kc {

// A (row-major n x n, symmetric) -> eigenvectors as columns of A; w -> eigenvalues
// (descending).
void sym_eig(int n, std::vector<double>& A, std::vector<double>& w) {
  std::vector<double> Q((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  std::vector<double> v(n), p(n), wv(n);
  auto a = [&](int r, int c) -> double& { return A[(size_t)r * n + c]; };
  // --- Householder tridiagonalisation: A = Q T Q^T
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;            // length of the column below the diagonal
    double nrm = 0.0;
    for (int i = 0; i < m; ++i) nrm = std::hypot(nrm, a(k + 1 + i, k));
    if (nrm == 0.0) continue;
    const double x0 = a(k + 1, k);
    const double alpha = x0 >= 0 ? -nrm : nrm;
    for (int i = 0; i < m; ++i) v[i] = a(k + 1 + i, k);
    v[0] -= alpha;
    double vv = 0.0;
    for (int i = 0; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    const double beta = 2.0 / vv;
    // p = beta * B v  (B the trailing block)
    for (int i = 0; i < m; ++i) {
      double s = 0.0;
      const double* row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
      for (int j = 0; j < m; ++j) s += row[j] * v[j];
      p[i] = beta * s;
    }
    double pv = 0.0;
    for (int i = 0; i < m; ++i) pv += p[i] * v[i];
    const double K = 0.5 * beta * pv;
    for (int i = 0; i < m; ++i) wv[i] = p[i] - K * v[i];
    for (int i = 0; i < m; ++i) {
      double* row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
      for (int j = 0; j < m; ++j) row[j] -= v[i] * wv[j] + wv[i] * v[j];
    }
    a(k + 1, k) = alpha;
    a(k, k + 1) = alpha;
    for (int i = 1; i < m; ++i) {
      a(k + 1 + i, k) = 0.0;
      a(k, k + 1 + i) = 0.0;
    }
    // Q <- Q (I - beta v v^T) on columns k+1..n-1
    for (int r = 0; r < n; ++r) {
      double* row = &Q[(size_t)r * n + (k + 1)];
      double s = 0.0;
      for (int i = 0; i < m; ++i) s += row[i] * v[i];
      s *= beta;
      for (int i = 0; i < m; ++i) row[i] -= s * v[i];
    }
  }
  std::vector<double> d(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = a(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = a(i + 1, i);
  // --- implicit QL on the tridiagonal (d, e), rotations accumulated into Q's columns
  const double eps = std::numeric_limits<double>::epsilon();
  for (int l = 0; l < n; ++l) {
    for (int iter = 0; iter < 200; ++iter) {
      int m = l;
      for (; m + 1 < n; ++m) {
        double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= eps * dd) break;
      }
      if (m == l) break;
      // shift from the leading 2x2 block
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
      double s = 1.0, c = 1.0, pacc = 0.0;
      int i = m - 1;
      bool early = false;
      for (; i >= l; --i) {
        double f = s * e[i];
        double b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= pacc;
          e[m] = 0.0;
          early = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - pacc;
        r = (d[i] - g) * s + 2.0 * c * b;
        pacc = s * r;
        d[i + 1] = g + pacc;
        g = c * r - b;
        for (int k = 0; k < n; ++k) {
          double* qk = &Q[(size_t)k * n];
          double t = qk[i + 1];
          qk[i + 1] = s * qk[i] + c * t;
          qk[i] = c * qk[i] - s * t;
        }
      }
      if (early) continue;
      d[l] -= pacc;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  // sort descending
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int x, int y) { return d[x] > d[y]; });
  w.resize(n);
  for (int c = 0; c < n; ++c) {
    w[c] = d[ord[c]];
    for (int r = 0; r < n; ++r) A[(size_t)r * n + c] = Q[(size_t)r * n + ord[c]];
  }
}

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
