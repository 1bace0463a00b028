// Pieces shared by the fine-propagator sources: where a system's start row comes from,
// the 2D face indexing, the float64 stencil and the stopping target of one implicit step.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace kc {

constexpr int kMaxRefinePasses = 12;
// A float32 pass reduces its residual only as far as the float64 target needs, times this
// margin (the 2-norm reduction that CG measures bounds the max-norm one only loosely; a
// pass that falls short is followed by another), and never beyond the tuned factor.
constexpr double kPassMargin = 0.1;

// start rows: if shift, the start of (m, s) is u0[m] (or 0) for s == 0 and start[m][s-1]
// otherwise (the parareal layout); else start[m][s]
struct StartRef {
  const double* start;
  const double* u0;
  bool shift;
  __device__ __forceinline__ const double* row(int64_t m, int s, int N, int64_t Nx) const {
    if (!shift) return start + ((int64_t)m * N + s) * Nx;
    if (s == 0) return u0 ? u0 + m * Nx : nullptr;
    return start + ((int64_t)m * N + (s - 1)) * Nx;
  }
};

// 2D face indexing: x-faces j (n+1) + f, then y-faces n (n+1) + f n + i
struct Grid2 {
  int n;
  int64_t nx;   // number of x-faces, n(n+1)
  __device__ __forceinline__ int64_t fW(int i, int j) const { return (int64_t)j * (n + 1) + i; }
  __device__ __forceinline__ int64_t fE(int i, int j) const { return (int64_t)j * (n + 1) + i + 1; }
  __device__ __forceinline__ int64_t fS(int i, int j) const { return nx + (int64_t)j * n + i; }
  __device__ __forceinline__ int64_t fN(int i, int j) const { return nx + (int64_t)(j + 1) * n + i; }
};

// Stopping target for the float64 residual of one implicit step: tol relative to the
// state size, but never below the rounding floor of forming that residual in float64,
// about eps * max_p d_p * |w|_inf (d_p the diagonal of I + tau A).
__device__ __forceinline__ double residual_target(double tol, double wmax, double tauf, double dmax) {
  return tol * (wmax + fabs(tauf)) + 8.0 * 2.220446049250313e-16 * dmax * wmax;
}

// (M v)_p - v_p = c * sum_faces a_f (v_p - v_q), float64, v read from global memory.
__device__ __forceinline__ double stencil64(const double* __restrict__ af, const double* __restrict__ v,
                                            const Grid2& g, int i, int j) {
  const int n = g.n;
  int64_t p = (int64_t)j * n + i;
  double vp = v[p];
  double vw = i > 0 ? v[p - 1] : 0.0;
  double ve = i < n - 1 ? v[p + 1] : 0.0;
  double vs = j > 0 ? v[p - n] : 0.0;
  double vn = j < n - 1 ? v[p + n] : 0.0;
  return af[g.fW(i, j)] * (vp - vw) + af[g.fE(i, j)] * (vp - ve) + af[g.fS(i, j)] * (vp - vs) +
         af[g.fN(i, j)] * (vp - vn);
}

}  // namespace kc
