// Input random field: KL eigenpairs of the exponential covariance and field synthesis.
//
// The input field of the diffusion coefficient is parameterised by a truncated KL
// expansion (Section 2, separated representation).  For sigma^2 exp(-|x-y|/l) on [0,1]
// the eigenpairs are known in closed form: with c = 1/l and s = x - 1/2 the roots w of
//   c cos(w/2) - w sin(w/2) = 0   (even modes, phi ~ cos(w s)),  w in (2m pi, (2m+1) pi)
//   w cos(w/2) + c sin(w/2) = 0   (odd modes,  phi ~ sin(w s)),  w in ((2m+1) pi, (2m+2) pi)
// give lambda = sigma^2 2c / (w^2 + c^2); the normalisations are 1/2 +- sin(w)/(2w).
// In 2D the covariance is the separable product, modes ordered by (-lambda, i+j, i).
#include <algorithm>
#include <cmath>
#include <tuple>

#include "common.h"

namespace kc {

namespace {

// Bisection to the last representable bit; f(lo) and f(hi) have opposite signs.
template <class F>
double bisect(F f, double lo, double hi) {
  double flo = f(lo);
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    double fm = f(mid);
    if ((fm < 0) == (flo < 0)) {
      lo = mid;
      flo = fm;
    } else {
      hi = mid;
    }
  }
  return 0.5 * (lo + hi);
}

struct Mode1D {
  double w, lam, norm;
  int parity;
};

std::vector<Mode1D> modes_1d(double corr_len, double sigma, int count) {
  const double c = 1.0 / corr_len;
  std::vector<Mode1D> out;
  for (int k = 0; (int)out.size() < count; ++k) {
    double lo = k * M_PI, hi = (k + 1) * M_PI;
    double w;
    if (k % 2 == 0)
      w = bisect([c](double x) { return c * std::cos(0.5 * x) - x * std::sin(0.5 * x); }, lo, hi);
    else
      w = bisect([c](double x) { return x * std::cos(0.5 * x) + c * std::sin(0.5 * x); }, lo, hi);
    Mode1D m;
    m.w = w;
    m.parity = k % 2;
    m.lam = sigma * sigma * 2.0 * c / (w * w + c * c);
    m.norm = std::sqrt(0.5 + (m.parity == 0 ? 1.0 : -1.0) * std::sin(w) / (2.0 * w));
    out.push_back(m);
  }
  return out;
}

inline double eval_mode(const Mode1D& m, double x) {
  double s = x - 0.5;
  return (m.parity == 0 ? std::cos(m.w * s) : std::sin(m.w * s)) / m.norm;
}

__global__ void field_synth_kernel(const double* __restrict__ phi, const double* __restrict__ sl,
                                   int d, int64_t nf, const double* __restrict__ xi, int64_t M,
                                   double* __restrict__ a, float* __restrict__ a32) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t m = blockIdx.y;
  if (f >= nf || m >= M) return;
  const double* x = xi + m * d;
  double s = 0.0;
  for (int k = 0; k < d; ++k) s += (sl[k] * x[k]) * phi[(int64_t)k * nf + f];
  const double v = exp(s);
  a[m * nf + f] = v;
  if (a32) a32[m * nf + f] = (float)v;   // round to nearest
}

}  // namespace

// lam [d] (descending) and phi [d][Fc] at the faces of the grid.
void field_kl_host(int dim, int n, int d, double corr_len, double sigma, std::vector<double>& lam,
                   std::vector<double>& phi) {
  const double h = 1.0 / (n + 1);
  const int64_t nf = n_faces(dim, n);
  lam.assign(d, 0.0);
  phi.assign((size_t)d * nf, 0.0);
  if (dim == 1) {
    auto ms = modes_1d(corr_len, sigma, d);
    for (int k = 0; k < d; ++k) {
      lam[k] = ms[k].lam;
      for (int f = 0; f <= n; ++f) phi[(size_t)k * nf + f] = eval_mode(ms[k], (f + 0.5) * h);
    }
    return;
  }
  const int m1 = d + 1;
  auto ms = modes_1d(corr_len, 1.0, m1);
  std::vector<std::tuple<double, int, int, int>> cand;
  for (int i = 0; i < m1; ++i)
    for (int j = 0; j < m1; ++j) cand.emplace_back(-(ms[i].lam * ms[j].lam), i + j, i, j);
  std::sort(cand.begin(), cand.end());
  const int64_t nx = (int64_t)n * (n + 1);
  for (int k = 0; k < d; ++k) {
    auto [negl, sum, i, j] = cand[k];
    (void)sum;
    lam[k] = sigma * sigma * (-negl);
    double* row = &phi[(size_t)k * nf];
    for (int jr = 0; jr < n; ++jr)          // x-faces: ((f+1/2)h, (jr+1)h)
      for (int f = 0; f <= n; ++f)
        row[jr * (n + 1) + f] = eval_mode(ms[i], (f + 0.5) * h) * eval_mode(ms[j], (jr + 1.0) * h);
    for (int f = 0; f <= n; ++f)            // y-faces: ((i+1)h, (f+1/2)h)
      for (int ic = 0; ic < n; ++ic)
        row[nx + f * n + ic] = eval_mode(ms[i], (ic + 1.0) * h) * eval_mode(ms[j], (f + 0.5) * h);
  }
}

void launch_field_synth(hipStream_t s, const double* phi, const double* sqrt_lam, int d,
                        int64_t nfaces, const double* xi, int64_t M, double* a, float* a32) {
  for (int64_t m0 = 0; m0 < M; m0 += 65535) {
    const int64_t Mc = std::min<int64_t>(65535, M - m0);
    dim3 grid((unsigned)((nfaces + 255) / 256), (unsigned)Mc);
    field_synth_kernel<<<grid, dim3(256), 0, s>>>(phi, sqrt_lam, d, nfaces, xi + m0 * d, Mc, a + m0 * nfaces,
                                                  a32 ? a32 + m0 * nfaces : nullptr);
    KC_LAUNCH_CHECK();
  }
}

}  // namespace kc
