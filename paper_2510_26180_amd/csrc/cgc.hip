// Diagonalised coarse grid correction (Section 3.2).
//
// The all-at-once coarse system (C_alpha (x) I + dT I (x) A) u = r of eq. matrix_NT is
// solved by the three steps of eq. three-steps, with the eigenvector matrix of C_alpha
// taken as V = Lambda^{-1} F_N (Lambda = diag(alpha^{s/N}), s = 0..N-1), the form that
// diagonalises C_alpha:
//   (a) p = F_N^* (Lambda r)       real FFT over the slice axis, float64
//   (b) (lambda_k I + dT A) q_k = p_k, lambda_k = 1 - alpha^{1/N} e^{-2 pi i k/N}
//   (c) u = Lambda^{-1} F_N q      inverse FFT, float64
// The input is real, so p_{N-k} = conj(p_k) and only k = 0..N/2 are solved.
// Layout: spectra are [M][N/2+1][Nx] complex128 (interleaved re, im).
#include <cmath>

#include <atomic>

#include "common.h"
#include "mg.h"
#include "reduce.h"

namespace kc {

namespace {

struct cd {
  double x, y;
};
__device__ __forceinline__ cd operator+(cd a, cd b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd operator-(cd a, cd b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cd operator*(cd a, cd b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ cd operator*(double s, cd a) { return {s * a.x, s * a.y}; }
__device__ __forceinline__ cd cdiv(cd a, cd b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, den = b.x + b.y * r;
    return {(a.x + a.y * r) / den, (a.y - a.x * r) / den};
  }
  double r = b.x / b.y, den = b.x * r + b.y;
  return {(a.x * r + a.y) / den, (a.y * r - a.x) / den};
}
__device__ __forceinline__ cd conj(cd a) { return {a.x, -a.y}; }

__device__ __forceinline__ int bitrev(int v, int logn) { return (int)(__brev((unsigned)v) >> (32 - logn)); }

// ---------------------------------------------------------------- defect
// D_s = (I + dT A)(F_s - U_s) for every slice: the right-hand side of the
// correction U^{k+1} - U^k of the all-at-once coarse system.
__global__ void defect_kernel(const double* __restrict__ a, int dim, int n, double cT,
                              const double* __restrict__ Fv, const double* __restrict__ U,
                              const uint8_t* __restrict__ active, int64_t M, int N,
                              double* __restrict__ D) {
  const int64_t Nx = dim == 1 ? n : (int64_t)n * n;
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t ms = blockIdx.y;   // m*N + s
  int64_t m = ms / N;
  if (p >= Nx) return;
  if (active && !active[m]) return;
  const double* f = Fv + ms * Nx;
  const double* u = U + ms * Nx;
  double e = f[p] - u[p];
  double acc;
  if (dim == 1) {
    const double* af = a + m * (n + 1);
    double ew = p > 0 ? f[p - 1] - u[p - 1] : 0.0;
    double ee = p < n - 1 ? f[p + 1] - u[p + 1] : 0.0;
    acc = af[p] * (e - ew) + af[p + 1] * (e - ee);
  } else {
    int64_t nx = (int64_t)n * (n + 1);
    const double* af = a + m * 2 * nx;
    int i = (int)(p % n), j = (int)(p / n);
    double ew = i > 0 ? f[p - 1] - u[p - 1] : 0.0;
    double ee = i < n - 1 ? f[p + 1] - u[p + 1] : 0.0;
    double es = j > 0 ? f[p - n] - u[p - n] : 0.0;
    double en = j < n - 1 ? f[p + n] - u[p + n] : 0.0;
    acc = af[(int64_t)j * (n + 1) + i] * (e - ew) + af[(int64_t)j * (n + 1) + i + 1] * (e - ee) +
          af[nx + (int64_t)j * n + i] * (e - es) + af[nx + (int64_t)(j + 1) * n + i] * (e - en);
  }
  D[ms * Nx + p] = e + cT * acc;
}

// ---------------------------------------------------------------- FFTs
// A work-group transforms C consecutive columns (m, x .. x + C - 1) along the slice axis:
// their N values live in LDS as [N][C] complex, thread t serves column t % C and takes
// every T-th butterfly of each radix-2 stage (T = threads per column), with a barrier
// between stages.  Consecutive threads hold consecutive columns, so every load and store
// of a slice row is one contiguous segment.
template <int C, int T>
__device__ __forceinline__ void fft_stages(cd* buf, const cd* tw, int N, int c, int r) {
  for (int len = 2; len <= N; len <<= 1) {
    const int half = len >> 1;
    const int stride = N / len;
    for (int b = r; b < N / 2; b += T) {
      const int k = b & (half - 1);
      const int i0 = (b - k) * 2 + k;            // start of the block + k
      const cd w = tw[k * stride];
      const cd u = buf[i0 * C + c];
      const cd v = buf[(i0 + half) * C + c] * w;
      buf[i0 * C + c] = u + v;
      buf[(i0 + half) * C + c] = u - v;
    }
    __syncthreads();
  }
}

template <int C, int T>
__global__ __launch_bounds__(C * T) void fft_forward_kernel(const double* __restrict__ r, int64_t Nx,
                                                            int N, int logn, double alpha,
                                                            const uint8_t* __restrict__ active,
                                                            double* __restrict__ spec) {
  extern __shared__ cd lds[];
  cd* buf = lds;                 // [N][C]
  cd* tw = lds + N * C;          // [N/2] e^{-2 pi i k / N}
  const int c = threadIdx.x % C, rr = threadIdx.x / C;
  const int64_t m = blockIdx.y;
  if (active && !active[m]) return;
  for (int k = threadIdx.x; k < N / 2; k += C * T) {
    double sv, cv;
    sincospi(-2.0 * k / N, &sv, &cv);
    tw[k] = {cv, sv};
  }
  const int64_t x = (int64_t)blockIdx.x * C + c;
  const bool ok = x < Nx;
  const double la = log(alpha) / N;
  const double* col = r + m * N * Nx + x;
  for (int s = rr; s < N; s += T) {
    const double sc = exp(la * s);   // alpha^{s/N}
    buf[bitrev(s, logn) * C + c] = {ok ? sc * col[(int64_t)s * Nx] : 0.0, 0.0};
  }
  __syncthreads();
  fft_stages<C, T>(buf, tw, N, c, rr);
  if (ok) {
    const double invsq = 1.0 / sqrt((double)N);
    const int K = N / 2 + 1;
    cd* out = (cd*)spec + m * K * Nx + x;
    for (int k = rr; k < K; k += T) out[(int64_t)k * Nx] = invsq * buf[k * C + c];
  }
}

// u_s = alpha^{-s/N} Re( N^{-1/2} sum_k e^{+2 pi i k s/N} Q_k ), Q_{N-k} = conj(Q_k).
// accumulate: u += result; maxima[m] = {max |result|, max |u_new|} as ordered bit patterns.
template <int C, int T>
__global__ __launch_bounds__(C * T) void fft_inverse_kernel(const double* __restrict__ spec,
                                                            int64_t Nx, int N, int logn,
                                                            double alpha,
                                                            const uint8_t* __restrict__ active,
                                                            double* __restrict__ u, int accumulate,
                                                            unsigned long long* __restrict__ maxima) {
  extern __shared__ cd lds[];
  cd* buf = lds;
  cd* tw = lds + N * C;          // e^{+2 pi i k / N}
  __shared__ double red[2][C * T / 64];
  const int c = threadIdx.x % C, rr = threadIdx.x / C;
  const int64_t m = blockIdx.y;
  if (active && !active[m]) return;
  for (int k = threadIdx.x; k < N / 2; k += C * T) {
    double sv, cv;
    sincospi(2.0 * k / N, &sv, &cv);
    tw[k] = {cv, sv};
  }
  const int64_t x = (int64_t)blockIdx.x * C + c;
  const bool ok = x < Nx;
  const int K = N / 2 + 1;
  const cd* in = (const cd*)spec + m * K * Nx + x;
  for (int k = rr; k < K; k += T) {
    const cd q = ok ? in[(int64_t)k * Nx] : cd{0.0, 0.0};
    buf[bitrev(k, logn) * C + c] = q;
    if (k > 0 && k < N - k) buf[bitrev(N - k, logn) * C + c] = conj(q);
  }
  __syncthreads();
  fft_stages<C, T>(buf, tw, N, c, rr);
  double cmax = 0.0, umax = 0.0;
  if (ok) {
    const double invsq = 1.0 / sqrt((double)N);
    const double la = -log(alpha) / N;
    double* col = u + m * N * Nx + x;
    for (int s = rr; s < N; s += T) {
      const double v = exp(la * s) * invsq * buf[s * C + c].x;
      double* dst = col + (int64_t)s * Nx;
      if (accumulate) {
        const double nu = *dst + v;
        *dst = nu;
        cmax = nanmax(cmax, fabs(v));
        umax = nanmax(umax, fabs(nu));
      } else {
        *dst = v;
      }
    }
  }
  if (maxima) {
    // non-negative doubles order like their bit patterns; one atomic per work-group
    cmax = wave_nanmax(cmax);
    umax = wave_nanmax(umax);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
      red[0][w] = cmax;
      red[1][w] = umax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int q = 1; q < C * T / 64; ++q) {
        cmax = nanmax(cmax, red[0][q]);
        umax = nanmax(umax, red[1][q]);
      }
      atomicMax(&maxima[2 * m], (unsigned long long)__double_as_longlong(cmax));
      atomicMax(&maxima[2 * m + 1], (unsigned long long)__double_as_longlong(umax));
    }
  }
}

// ---------------------------------------------------------------- step (b), 1D
// Complex tridiagonal (Thomas) solve per (m, k): (lambda_k I + dT A) q = p, in place.
// Re(lambda_k) > 0 and A is an M-matrix, so the matrix is diagonally dominant and
// elimination without pivoting is stable.
__global__ void shifted_tri_kernel(const double* __restrict__ a, int n, double cT, int N,
                                   double alpha, const uint8_t* __restrict__ active, int64_t M,
                                   double* __restrict__ spec, double* __restrict__ scratch) {
  const int K = N / 2 + 1;
  int64_t sys = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t m = sys / K;
  int k = (int)(sys % K);
  if (m >= M) return;
  if (active && !active[m]) return;
  double sv, cv;
  sincospi(-2.0 * k / N, &sv, &cv);
  const double an = exp(log(alpha) / N);
  const cd lam = {1.0 - an * cv, -an * sv};
  const double* af = a + m * (n + 1);
  cd* q = (cd*)spec + sys * n;
  cd* cp = (cd*)scratch + sys * n;
  cd prevc = {0.0, 0.0};
  cd prevd = {0.0, 0.0};
  for (int i = 0; i < n; ++i) {
    double aw = af[i], ae = af[i + 1];
    cd diag = {lam.x + cT * (aw + ae), lam.y};
    double lo = i > 0 ? -cT * aw : 0.0;
    double up = i < n - 1 ? -cT * ae : 0.0;
    cd den = diag - lo * prevc;
    cd c = cdiv(cd{up, 0.0}, den);
    cd d = cdiv(q[i] - lo * prevd, den);
    cp[i] = c;
    q[i] = d;
    prevc = c;
    prevd = d;
  }
  for (int i = n - 2; i >= 0; --i) q[i] = q[i] - cp[i] * q[i + 1];
}

// ---------------------------------------------------------------- step (b), 2D
// Jacobi-preconditioned COCG (conjugate orthogonal CG: the unconjugated bilinear form
// suits the complex-symmetric matrix lambda_k I + dT A) in complex128, one work-group
// per (m, k) system, vectors streamed through per-system scratch; x is the spectrum.
constexpr int kCocgThreads = 256;

__device__ __forceinline__ cd shifted_apply(const double* __restrict__ af, const cd* __restrict__ v,
                                            int n, int64_t nx, double cT, cd lam, int i, int j) {
  int64_t p = (int64_t)j * n + i;
  cd vp = v[p];
  cd zero = {0.0, 0.0};
  cd vw = i > 0 ? v[p - 1] : zero;
  cd ve = i < n - 1 ? v[p + 1] : zero;
  cd vs = j > 0 ? v[p - n] : zero;
  cd vn = j < n - 1 ? v[p + n] : zero;
  cd acc = af[(int64_t)j * (n + 1) + i] * (vp - vw) + af[(int64_t)j * (n + 1) + i + 1] * (vp - ve) +
           af[nx + (int64_t)j * n + i] * (vp - vs) + af[nx + (int64_t)(j + 1) * n + i] * (vp - vn);
  return lam * vp + cT * acc;
}

__global__ __launch_bounds__(kCocgThreads) void cocg_kernel(const double* __restrict__ a, int n,
                                                            double cT, int N, double alpha,
                                                            double rtol, int maxit,
                                                            const uint8_t* __restrict__ active,
                                                            double* __restrict__ spec,
                                                            double* __restrict__ scr,
                                                            int* __restrict__ flag,
                                                            unsigned long long* __restrict__ cnt) {
  __shared__ double slots[4 * (kCocgThreads / 64)];
  const int K = N / 2 + 1;
  const int64_t sys = blockIdx.x;
  const int64_t m = sys / K;
  const int k = (int)(sys % K);
  if (active && !active[m]) return;
  const int64_t Nx = (int64_t)n * n;
  const int64_t nx = (int64_t)n * (n + 1);
  const double* af = a + m * 2 * nx;
  double sv, cv;
  sincospi(-2.0 * k / N, &sv, &cv);
  const double an = exp(log(alpha) / N);
  const cd lam = {1.0 - an * cv, -an * sv};
  cd* x = (cd*)spec + sys * Nx;
  cd* R = (cd*)scr + sys * 3 * Nx;
  cd* P = R + Nx;
  cd* Q = P + Nx;
  // x0 = 0: r = b, z = D^{-1} r
  double acc[3] = {0.0, 0.0, 0.0};   // rz (re, im), |r|^2
  const bool mx3[3] = {false, false, false};
  for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
    int i = (int)(p % n), j = (int)(p / n);
    cd r = x[p];
    double sa = af[(int64_t)j * (n + 1) + i] + af[(int64_t)j * (n + 1) + i + 1] + af[nx + (int64_t)j * n + i] +
                af[nx + (int64_t)(j + 1) * n + i];
    cd d = {lam.x + cT * sa, lam.y};
    cd z = cdiv(r, d);
    R[p] = r;
    P[p] = z;
    x[p] = {0.0, 0.0};
    cd rz = r * z;
    acc[0] += rz.x;
    acc[1] += rz.y;
    acc[2] += r.x * r.x + r.y * r.y;
  }
  block_reduce<3>(acc, mx3, slots);
  cd rz = {acc[0], acc[1]};
  const double bnorm2 = acc[2];
  double rnorm2 = acc[2];
  const double stop2 = rtol * rtol * bnorm2;
  int it = 0;
  while (rnorm2 > stop2 && it < maxit) {
    double pq2[2] = {0.0, 0.0};
    const bool mx2[2] = {false, false};
    for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
      int i = (int)(p % n), j = (int)(p / n);
      cd q = shifted_apply(af, P, n, nx, cT, lam, i, j);
      Q[p] = q;
      cd pq = P[p] * q;
      pq2[0] += pq.x;
      pq2[1] += pq.y;
    }
    block_reduce<2>(pq2, mx2, slots);
    const cd alph = cdiv(rz, cd{pq2[0], pq2[1]});
    double acc2[3] = {0.0, 0.0, 0.0};
    for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
      int i = (int)(p % n), j = (int)(p / n);
      x[p] = x[p] + alph * P[p];
      cd r = R[p] - alph * Q[p];
      R[p] = r;
      double sa = af[(int64_t)j * (n + 1) + i] + af[(int64_t)j * (n + 1) + i + 1] + af[nx + (int64_t)j * n + i] +
                  af[nx + (int64_t)(j + 1) * n + i];
      cd z = cdiv(r, cd{lam.x + cT * sa, lam.y});
      Q[p] = z;   // reuse Q for z
      cd rzp = r * z;
      acc2[0] += rzp.x;
      acc2[1] += rzp.y;
      acc2[2] += r.x * r.x + r.y * r.y;
    }
    block_reduce<3>(acc2, mx3, slots);
    const cd rzn = {acc2[0], acc2[1]};
    const cd beta = cdiv(rzn, rz);
    rz = rzn;
    rnorm2 = acc2[2];
    for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) P[p] = Q[p] + beta * P[p];
    __syncthreads();
    ++it;
  }
  if (threadIdx.x == 0) {
    if (rnorm2 > stop2) atomicOr(flag, 1);
    atomicAdd(&cnt[0], (unsigned long long)it);
    atomicAdd(&cnt[2], 1ull);
    atomicMax(&cnt[3], (unsigned long long)it);
  }
}

// ------------------------------------------------ step (b), 2D, CU-resident
// For grids up to 64x64 (the whole system's Krylov state fits one CU's registers; a
// 128x128 complex system does not), the same shifted systems solved on one CU each: float32 complex COCG on the
// real-Jacobi-scaled matrix  D^{-1/2} (lambda I + dT A) D^{-1/2} = diag(1 + i theta) - S,
// D = Re(lambda) + dT diag(A), theta_p = Im(lambda) / D_p, S the scaled (real) face
// couplings, refined in float64: the complex128 residual p - (lambda I + dT A) q is kept
// in global memory, each pass solves for a correction in float32 (Krylov state in
// registers, the correction accumulated in an LDS tile), adds it to q in float64 and
// updates the residual, until |res|_2 <= rtol |p|_2.

// D_r^{-1/2} of the shifted systems mk0 .. mk0 + gridDim.y - 1, stored from dr (row of system
// mk0 first)
__global__ void shift_dinv_kernel(const double* __restrict__ a, int n, double cT, int N, double alpha,
                                  int64_t M, double* __restrict__ dr, int64_t mk0 = 0) {
  const int K = N / 2 + 1;
  const int64_t Nx = (int64_t)n * n;
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t mk = mk0 + blockIdx.y;
  if (p >= Nx || mk >= M * K) return;
  int64_t m = mk / K;
  int k = (int)(mk % K);
  double sv, cv;
  sincospi(-2.0 * k / N, &sv, &cv);
  const double lre = 1.0 - exp(log(alpha) / N) * cv;
  const int64_t nx = (int64_t)n * (n + 1);
  const double* af = a + m * 2 * nx;
  int i = (int)(p % n), j = (int)(p / n);
  double sa = af[(int64_t)j * (n + 1) + i] + af[(int64_t)j * (n + 1) + i + 1] + af[nx + (int64_t)j * n + i] +
              af[nx + (int64_t)(j + 1) * n + i];
  dr[(mk - mk0) * Nx + p] = 1.0 / sqrt(lre + cT * sa);
}

template <int CTRL>
__device__ __forceinline__ float dppf_c(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
__device__ __forceinline__ float wsum_dpp(float v) {
  v += dppf_c<0xB1>(v);
  v += dppf_c<0x4E>(v);
  v += dppf_c<0x141>(v);
  v += dppf_c<0x140>(v);
  const int iv = __builtin_bit_cast(int, v);
  return (__builtin_bit_cast(float, __builtin_amdgcn_readlane(iv, 0)) +
          __builtin_bit_cast(float, __builtin_amdgcn_readlane(iv, 16))) +
         (__builtin_bit_cast(float, __builtin_amdgcn_readlane(iv, 32)) +
          __builtin_bit_cast(float, __builtin_amdgcn_readlane(iv, 48)));
}
template <int NW, int K>
__device__ __forceinline__ void block_sum_fk(float (&v)[K], float* slots, int lane, int wave) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wsum_dpp(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) slots[k * NW + wave] = v[k];
  }
  __syncthreads();
  // the NW wave sums by the same row butterfly in lanes 0..NW-1, read back as a scalar
#pragma unroll
  for (int k = 0; k < K; ++k) {
    float x = lane < NW ? slots[k * NW + lane] : 0.f;
    x += dppf_c<0xB1>(x);
    x += dppf_c<0x4E>(x);
    x += dppf_c<0x141>(x);
    x += dppf_c<0x140>(x);
    v[k] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 0));
  }
}

struct cf {
  float x, y;
};
__device__ __forceinline__ cf cf_div(cf a, cf b) {
  float den = b.x * b.x + b.y * b.y;
  return {(a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den};
}

template <int NW, int CPL, int RPW>
__global__ __launch_bounds__(64 * NW) void cocg_resident_kernel(
    const double* __restrict__ a, const double* __restrict__ dinvr, int n, double cT, int N, double alpha,
    double rtol, float inner_rtol, int maxit, const uint8_t* __restrict__ active, double* __restrict__ spec,
    double* __restrict__ resbuf, int* __restrict__ flag, unsigned long long* __restrict__ cnt) {
  constexpr int ROWW = 64 * CPL;
  extern __shared__ float2 xs[];                 // [n*n] complex64 correction / staging
  __shared__ float2 htop[(NW - 1) * ROWW];       // boundary b: NS(row 0 of wave b+1) * P
  __shared__ float2 hbot[(NW - 1) * ROWW];       // boundary b: last row of wave b
  __shared__ float fsl[2][3 * NW];
  __shared__ double dsl[4 * NW];
  const int K = N / 2 + 1;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t sys = blockIdx.x;
  const int64_t m = sys / K;
  const int k = (int)(sys % K);
  if (active && !active[m]) return;
  const int64_t Nx = (int64_t)n * n;
  const int64_t nx = (int64_t)n * (n + 1);
  const double* af = a + m * 2 * nx;
  const double* dr = dinvr + sys * Nx;
  double2* q = (double2*)spec + sys * Nx;
  double2* res = (double2*)resbuf + sys * Nx;
  double sv, cv;
  sincospi(-2.0 * k / N, &sv, &cv);
  const double an = exp(log(alpha) / N);
  const double lre = 1.0 - an * cv, lim = -an * sv;
  const int j0 = wave * RPW, i0 = lane * CPL;

  float EW[RPW][CPL], NS[RPW][CPL], TH[RPW][CPL];
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    const int j = j0 + r;
#pragma unroll
    for (int t = 0; t < CPL; ++t) {
      const int i = i0 + t;
      const bool in = (j < n && i < n);
      const int64_t p = (int64_t)j * n + i;
      EW[r][t] = (in && i >= 1) ? (float)(cT * af[(int64_t)j * (n + 1) + i] * dr[p - 1] * dr[p]) : 0.f;
      NS[r][t] = (in && j >= 1) ? (float)(cT * af[nx + (int64_t)j * n + i] * dr[p - n] * dr[p]) : 0.f;
      TH[r][t] = in ? (float)(lim * dr[p] * dr[p]) : 0.f;
    }
  }
  // res = p, q = 0, |p|_2^2 and the scale of the next float32 right-hand side
  double bn[2] = {0.0, 0.0};
  const bool sm[2] = {false, true};
  for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
    double2 v = q[p];
    res[p] = v;
    q[p] = make_double2(0.0, 0.0);
    bn[0] += v.x * v.x + v.y * v.y;
    bn[1] = nanmax(bn[1], dr[p] * fmax(fabs(v.x), fabs(v.y)));
  }
  block_reduce<2>(bn, sm, dsl);
  const double stop2 = rtol * rtol * bn[0];
  double rn2 = bn[0];
  // float32 right-hand sides are normalised by their max so that tiny late-pass
  // residuals do not underflow
  double sig = bn[1];
  unsigned long long tot_it = 0, max_it = 0;
  int pass = 0;
  float2 R[RPW][CPL], P[RPW][CPL];
  while (rn2 > stop2 && sig > 0.0 && pass < 12) {
    const double isig = 1.0 / sig;
    // stage D^{-1/2} res / sig as complex64 through LDS
#pragma unroll 1
    for (int kk = 0; kk < RPW * CPL; ++kk) {
      const int j = j0 + kk / CPL, i = i0 + kk % CPL;
      if (j < n && i < n) {
        const int64_t p = (int64_t)j * n + i;
        const double2 v = res[p];
        xs[p] = make_float2((float)(isig * dr[p] * v.x), (float)(isig * dr[p] * v.y));
      }
    }
    __syncthreads();
    float acc3[3] = {0.f, 0.f, 0.f};   // r.r (re, im), |r|^2
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int j = j0 + r;
#pragma unroll
      for (int t = 0; t < CPL; ++t) {
        const int i = i0 + t;
        float2 v = (j < n && i < n) ? xs[j * n + i] : make_float2(0.f, 0.f);
        R[r][t] = v;
        P[r][t] = v;
        acc3[0] += v.x * v.x - v.y * v.y;
        acc3[1] += 2.f * v.x * v.y;
        acc3[2] += v.x * v.x + v.y * v.y;
      }
    }
    __syncthreads();   // everyone has read the staged right-hand side
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int j = j0 + r;
#pragma unroll
      for (int t = 0; t < CPL; ++t) {
        const int i = i0 + t;
        if (j < n && i < n) xs[j * n + i] = make_float2(0.f, 0.f);
      }
    }
    block_sum_fk<NW, 3>(acc3, fsl[1], lane, wave);
    cf rz = {acc3[0], acc3[1]};
    float rr = acc3[2];
    const float stop_in = inner_rtol * inner_rtol * rr;
    int it = 0;
    // a pass restarts from the true float64 residual after a few times n iterations
    // (COCG can stagnate near a breakdown of its unconjugated form)
    const int cap = maxit < 4 * n + 200 ? maxit : 4 * n + 200;
    bool bad = false;
    while (rr > stop_in && it < cap) {
      // halos of P
#pragma unroll
      for (int t = 0; t < CPL; ++t) {
        if (wave < NW - 1) hbot[wave * ROWW + lane * CPL + t] = P[RPW - 1][t];
        if (wave > 0)
          htop[(wave - 1) * ROWW + lane * CPL + t] = make_float2(NS[0][t] * P[0][t].x, NS[0][t] * P[0][t].y);
      }
      __syncthreads();
      // pass 1: pq = sum p (M p) (unconjugated)
      float pq2[2] = {0.f, 0.f};
#pragma unroll
      for (int pass_mv = 0; pass_mv < 2; ++pass_mv) {
        cf alph = {0.f, 0.f};
        if (pass_mv == 1) {
          block_sum_fk<NW, 2>(pq2, fsl[0], lane, wave);
          alph = cf_div(rz, cf{pq2[0], pq2[1]});
        }
        float racc[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
          const float wvx = dppf_c<0x138>(P[r][CPL - 1].x), wvy = dppf_c<0x138>(P[r][CPL - 1].y);
          const float epx = dppf_c<0x130>(EW[r][0] * P[r][0].x), epy = dppf_c<0x130>(EW[r][0] * P[r][0].y);
#pragma unroll
          for (int t = 0; t < CPL; ++t) {
            const float2 pv = P[r][t];
            float qx = pv.x - TH[r][t] * pv.y, qy = pv.y + TH[r][t] * pv.x;
            const float lx = (t == 0) ? wvx : P[r][t - 1].x, ly = (t == 0) ? wvy : P[r][t - 1].y;
            qx = fmaf(-EW[r][t], lx, qx);
            qy = fmaf(-EW[r][t], ly, qy);
            if (t == CPL - 1) {
              qx -= epx;
              qy -= epy;
            } else {
              qx = fmaf(-EW[r][t + 1], P[r][t + 1].x, qx);
              qy = fmaf(-EW[r][t + 1], P[r][t + 1].y, qy);
            }
            float2 dn, up;
            if (r == 0)
              dn = (wave > 0) ? hbot[(wave - 1) * ROWW + lane * CPL + t] : make_float2(0.f, 0.f);
            else
              dn = P[r - 1][t];
            qx = fmaf(-NS[r][t], dn.x, qx);
            qy = fmaf(-NS[r][t], dn.y, qy);
            if (r == RPW - 1) {
              up = (wave < NW - 1) ? htop[wave * ROWW + lane * CPL + t] : make_float2(0.f, 0.f);
              qx -= up.x;
              qy -= up.y;
            } else {
              qx = fmaf(-NS[r + 1][t], P[r + 1][t].x, qx);
              qy = fmaf(-NS[r + 1][t], P[r + 1][t].y, qy);
            }
            if (pass_mv == 0) {
              pq2[0] += pv.x * qx - pv.y * qy;
              pq2[1] += pv.x * qy + pv.y * qx;
            } else {
              float2 rv = R[r][t];
              rv.x -= alph.x * qx - alph.y * qy;
              rv.y -= alph.x * qy + alph.y * qx;
              R[r][t] = rv;
            }
          }
        }
        if (pass_mv == 1) {
          // correction tile X += alpha P, and the new residual's dot products
#pragma unroll
          for (int r = 0; r < RPW; ++r) {
            const int j = j0 + r;
#pragma unroll
            for (int t = 0; t < CPL; ++t) {
              const int i = i0 + t;
              const float2 pv = P[r][t], rv = R[r][t];
              if (j < n && i < n) {
                float2 xv = xs[j * n + i];
                xv.x += alph.x * pv.x - alph.y * pv.y;
                xv.y += alph.x * pv.y + alph.y * pv.x;
                xs[j * n + i] = xv;
              }
              racc[0] += rv.x * rv.x - rv.y * rv.y;
              racc[1] += 2.f * rv.x * rv.y;
              racc[2] += rv.x * rv.x + rv.y * rv.y;
            }
          }
        }
        if (pass_mv == 1) {
          block_sum_fk<NW, 3>(racc, fsl[1], lane, wave);
          const cf rzn = {racc[0], racc[1]};
          const cf beta = cf_div(rzn, rz);
          rz = rzn;
          rr = racc[2];
          if (!(rr < 3.0e38f) || !(fabsf(rz.x) + fabsf(rz.y) < 3.0e38f)) bad = true;
#pragma unroll
          for (int r = 0; r < RPW; ++r)
#pragma unroll
            for (int t = 0; t < CPL; ++t) {
              const float2 pv = P[r][t], rv = R[r][t];
              P[r][t] = make_float2(rv.x + beta.x * pv.x - beta.y * pv.y, rv.y + beta.x * pv.y + beta.y * pv.x);
            }
        }
      }
      ++it;
      if (bad) break;
    }
    tot_it += it;
    max_it = it > (int)max_it ? it : max_it;
    if (bad) {   // keep the last good q and report
      if (threadIdx.x == 0) atomicOr(flag, 1);
      break;
    }
    __syncthreads();   // correction tile complete
    // float64: e = sig D^{-1/2} X; res -= (lambda I + dT A) e; q += e
    double acc[2] = {0.0, 0.0};
#pragma unroll 1
    for (int kk = 0; kk < RPW * CPL; ++kk) {
      const int j = j0 + kk / CPL, i = i0 + kk % CPL;
      if (j < n && i < n) {
        const int64_t p = (int64_t)j * n + i;
        const float2 xp = xs[p];
        const double ex = sig * dr[p] * xp.x, ey = sig * dr[p] * xp.y;
        double sx = 0.0, sy = 0.0;
        const double aW = af[(int64_t)j * (n + 1) + i], aE = af[(int64_t)j * (n + 1) + i + 1];
        const double aS = af[nx + (int64_t)j * n + i], aN = af[nx + (int64_t)(j + 1) * n + i];
        {
          double nxv = 0.0, nyv = 0.0;
          if (i > 0) { const float2 v = xs[p - 1]; nxv = sig * dr[p - 1] * v.x; nyv = sig * dr[p - 1] * v.y; }
          sx += aW * (ex - nxv); sy += aW * (ey - nyv);
        }
        {
          double nxv = 0.0, nyv = 0.0;
          if (i < n - 1) { const float2 v = xs[p + 1]; nxv = sig * dr[p + 1] * v.x; nyv = sig * dr[p + 1] * v.y; }
          sx += aE * (ex - nxv); sy += aE * (ey - nyv);
        }
        {
          double nxv = 0.0, nyv = 0.0;
          if (j > 0) { const float2 v = xs[p - n]; nxv = sig * dr[p - n] * v.x; nyv = sig * dr[p - n] * v.y; }
          sx += aS * (ex - nxv); sy += aS * (ey - nyv);
        }
        {
          double nxv = 0.0, nyv = 0.0;
          if (j < n - 1) { const float2 v = xs[p + n]; nxv = sig * dr[p + n] * v.x; nyv = sig * dr[p + n] * v.y; }
          sx += aN * (ex - nxv); sy += aN * (ey - nyv);
        }
        const double mex = lre * ex - lim * ey + cT * sx;
        const double mey = lre * ey + lim * ex + cT * sy;
        double2 rv = res[p];
        rv.x -= mex;
        rv.y -= mey;
        res[p] = rv;
        double2 qv = q[p];
        qv.x += ex;
        qv.y += ey;
        q[p] = qv;
        acc[0] += rv.x * rv.x + rv.y * rv.y;
        acc[1] = nanmax(acc[1], dr[p] * fmax(fabs(rv.x), fabs(rv.y)));
      }
    }
    block_reduce<2>(acc, sm, dsl);
    rn2 = acc[0];
    sig = acc[1];
    ++pass;
  }
  if (threadIdx.x == 0) {
    if (rn2 > stop2) {
      atomicOr(flag, 1);
      atomicAdd(&cnt[5], 1ull);
    }
    atomicAdd(&cnt[0], tot_it);
    atomicAdd(&cnt[1], (unsigned long long)pass);
    atomicAdd(&cnt[2], 1ull);
    atomicMax(&cnt[3], max_it);
  }
}

// Streaming variant for grids too large for one CU's registers: one work-group per
// (m, k) system, complex64 Krylov vectors and float32 scaled couplings in per-system
// global scratch, with the same float64 residual refinement as above.
struct Cocg32Scratch {
  float2 *X, *R, *P, *Q;   // [Nx] each
  float *cw, *cs, *th;     // west / south coupling, imaginary diagonal
};

__global__ __launch_bounds__(512) void cocg32_stream_kernel(
    const double* __restrict__ a, const double* __restrict__ dinvr, int n, double cT, int N, double alpha,
    double rtol, float inner_rtol, int maxit, const uint8_t* __restrict__ active, double* __restrict__ spec,
    double* __restrict__ resbuf, float* __restrict__ scr, int* __restrict__ flag,
    unsigned long long* __restrict__ cnt) {
  constexpr int NW = 8;
  __shared__ float fsl[2][3 * NW];
  __shared__ double dsl[4 * NW];
  const int K = N / 2 + 1;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t sys = blockIdx.x;
  const int64_t m = sys / K;
  const int k = (int)(sys % K);
  if (active && !active[m]) return;
  const int64_t Nx = (int64_t)n * n;
  const int64_t nx = (int64_t)n * (n + 1);
  const double* af = a + m * 2 * nx;
  const double* dr = dinvr + sys * Nx;
  double2* q = (double2*)spec + sys * Nx;
  double2* res = (double2*)resbuf + sys * Nx;
  float* base = scr + sys * 11 * Nx;
  float2* X = (float2*)base;
  float2* R = X + Nx;
  float2* P = R + Nx;
  float2* Q = P + Nx;
  float* cw = (float*)(Q + Nx);
  float* cs = cw + Nx;
  float* th = cs + Nx;
  double sv, cv;
  sincospi(-2.0 * k / N, &sv, &cv);
  const double an = exp(log(alpha) / N);
  const double lre = 1.0 - an * cv, lim = -an * sv;

  double bn[2] = {0.0, 0.0};
  const bool sm[2] = {false, true};
  for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
    const int i = (int)(p % n), j = (int)(p / n);
    cw[p] = i >= 1 ? (float)(cT * af[(int64_t)j * (n + 1) + i] * dr[p - 1] * dr[p]) : 0.f;
    cs[p] = j >= 1 ? (float)(cT * af[nx + (int64_t)j * n + i] * dr[p - n] * dr[p]) : 0.f;
    th[p] = (float)(lim * dr[p] * dr[p]);
    const double2 v = q[p];
    res[p] = v;
    q[p] = make_double2(0.0, 0.0);
    bn[0] += v.x * v.x + v.y * v.y;
    bn[1] = nanmax(bn[1], dr[p] * fmax(fabs(v.x), fabs(v.y)));
  }
  block_reduce<2>(bn, sm, dsl);
  const double stop2 = rtol * rtol * bn[0];
  double rn2 = bn[0];
  double sig = bn[1];
  unsigned long long tot_it = 0, max_it = 0;
  int pass = 0;
  while (rn2 > stop2 && sig > 0.0 && pass < 12) {
    const double isig = 1.0 / sig;
    float acc3[3] = {0.f, 0.f, 0.f};
    for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
      const double2 rv = res[p];
      const float2 v = make_float2((float)(isig * dr[p] * rv.x), (float)(isig * dr[p] * rv.y));
      R[p] = v;
      P[p] = v;
      X[p] = make_float2(0.f, 0.f);
      acc3[0] += v.x * v.x - v.y * v.y;
      acc3[1] += 2.f * v.x * v.y;
      acc3[2] += v.x * v.x + v.y * v.y;
    }
    block_sum_fk<NW, 3>(acc3, fsl[1], lane, wave);   // its barrier also publishes P
    cf rz = {acc3[0], acc3[1]};
    float rr = acc3[2];
    const float stop_in = inner_rtol * inner_rtol * rr;
    int it = 0;
    // a pass restarts from the true float64 residual after a few times n iterations
    // (COCG can stagnate near a breakdown of its unconjugated form)
    const int cap = maxit < 4 * n + 200 ? maxit : 4 * n + 200;
    bool bad = false;
    while (rr > stop_in && it < cap) {
      float pq2[2] = {0.f, 0.f};
      for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
        const int i = (int)(p % n), j = (int)(p / n);
        const float2 pv = P[p];
        const float2 zero = make_float2(0.f, 0.f);
        const float2 lw = i > 0 ? P[p - 1] : zero, le = i < n - 1 ? P[p + 1] : zero;
        const float2 ls = j > 0 ? P[p - n] : zero, ln = j < n - 1 ? P[p + n] : zero;
        const float ce = i < n - 1 ? cw[p + 1] : 0.f, cn = j < n - 1 ? cs[p + n] : 0.f;
        const float c0 = cw[p], c1 = cs[p], t0 = th[p];
        float qx = pv.x - t0 * pv.y - c0 * lw.x - ce * le.x - c1 * ls.x - cn * ln.x;
        float qy = pv.y + t0 * pv.x - c0 * lw.y - ce * le.y - c1 * ls.y - cn * ln.y;
        Q[p] = make_float2(qx, qy);
        pq2[0] += pv.x * qx - pv.y * qy;
        pq2[1] += pv.x * qy + pv.y * qx;
      }
      block_sum_fk<NW, 2>(pq2, fsl[0], lane, wave);
      const cf al = cf_div(rz, cf{pq2[0], pq2[1]});
      float racc[3] = {0.f, 0.f, 0.f};
      for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
        const float2 pv = P[p], qv = Q[p];
        float2 xv = X[p], rv = R[p];
        xv.x += al.x * pv.x - al.y * pv.y;
        xv.y += al.x * pv.y + al.y * pv.x;
        rv.x -= al.x * qv.x - al.y * qv.y;
        rv.y -= al.x * qv.y + al.y * qv.x;
        X[p] = xv;
        R[p] = rv;
        racc[0] += rv.x * rv.x - rv.y * rv.y;
        racc[1] += 2.f * rv.x * rv.y;
        racc[2] += rv.x * rv.x + rv.y * rv.y;
      }
      block_sum_fk<NW, 3>(racc, fsl[1], lane, wave);
      const cf rzn = {racc[0], racc[1]};
      const cf be = cf_div(rzn, rz);
      rz = rzn;
      rr = racc[2];
      if (!(rr < 3.0e38f) || !(fabsf(rz.x) + fabsf(rz.y) < 3.0e38f)) bad = true;
      for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
        const float2 pv = P[p], rv = R[p];
        P[p] = make_float2(rv.x + be.x * pv.x - be.y * pv.y, rv.y + be.x * pv.y + be.y * pv.x);
      }
      __syncthreads();
      ++it;
      if (bad) break;
    }
    tot_it += it;
    max_it = it > (int)max_it ? it : max_it;
    if (bad) {   // keep the last good q and report
      if (threadIdx.x == 0) atomicOr(flag, 1);
      break;
    }
    double acc[2] = {0.0, 0.0};
    for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
      const int i = (int)(p % n), j = (int)(p / n);
      const float2 xp = X[p];
      const double ex = sig * dr[p] * xp.x, ey = sig * dr[p] * xp.y;
      double sx = 0.0, sy = 0.0;
      const double aW = af[(int64_t)j * (n + 1) + i], aE = af[(int64_t)j * (n + 1) + i + 1];
      const double aS = af[nx + (int64_t)j * n + i], aN = af[nx + (int64_t)(j + 1) * n + i];
      double nxv, nyv;
      nxv = nyv = 0.0;
      if (i > 0) { const float2 v = X[p - 1]; nxv = sig * dr[p - 1] * v.x; nyv = sig * dr[p - 1] * v.y; }
      sx += aW * (ex - nxv); sy += aW * (ey - nyv);
      nxv = nyv = 0.0;
      if (i < n - 1) { const float2 v = X[p + 1]; nxv = sig * dr[p + 1] * v.x; nyv = sig * dr[p + 1] * v.y; }
      sx += aE * (ex - nxv); sy += aE * (ey - nyv);
      nxv = nyv = 0.0;
      if (j > 0) { const float2 v = X[p - n]; nxv = sig * dr[p - n] * v.x; nyv = sig * dr[p - n] * v.y; }
      sx += aS * (ex - nxv); sy += aS * (ey - nyv);
      nxv = nyv = 0.0;
      if (j < n - 1) { const float2 v = X[p + n]; nxv = sig * dr[p + n] * v.x; nyv = sig * dr[p + n] * v.y; }
      sx += aN * (ex - nxv); sy += aN * (ey - nyv);
      const double mex = lre * ex - lim * ey + cT * sx;
      const double mey = lre * ey + lim * ex + cT * sy;
      double2 rv = res[p];
      rv.x -= mex;
      rv.y -= mey;
      res[p] = rv;
      double2 qv = q[p];
      qv.x += ex;
      qv.y += ey;
      q[p] = qv;
      acc[0] += rv.x * rv.x + rv.y * rv.y;
      acc[1] = nanmax(acc[1], dr[p] * fmax(fabs(rv.x), fabs(rv.y)));
    }
    block_reduce<2>(acc, sm, dsl);
    rn2 = acc[0];
    sig = acc[1];
    ++pass;
  }
  if (threadIdx.x == 0) {
    if (rn2 > stop2) {
      atomicOr(flag, 1);
      atomicAdd(&cnt[5], 1ull);
    }
    atomicAdd(&cnt[0], tot_it);
    atomicAdd(&cnt[1], (unsigned long long)pass);
    atomicAdd(&cnt[2], 1ull);
    atomicMax(&cnt[3], max_it);
  }
}

// ---------------------------------------------------------------- multigrid-preconditioned COCG
// Float32 COCG on the Jacobi-scaled shifted system L = (1 + i theta) I - C, preconditioned
// by one aggregation-multigrid V-cycle (mg.h), inside the same float64 residual refinement
// as the kernels above.  System scratch: X, R, P, Q (complex, n^2 each), then the levels.
template <int NW, int WPE>
__global__ __launch_bounds__(64 * NW, WPE) void cocg_mg_kernel(
    const double* __restrict__ a, const double* __restrict__ dinvr, int n, double cT, int N, double alpha,
    double rtol, float inner_rtol, int maxit, const uint8_t* __restrict__ active, double* __restrict__ spec,
    double* __restrict__ resbuf, float* __restrict__ scr, MgLevels h, int* __restrict__ flag,
    unsigned long long* __restrict__ cnt, int64_t sys0) {
  __shared__ float fsl[2][3 * NW];
  __shared__ double dsl[4 * NW];
  const int K = N / 2 + 1;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  // system sys0 + b of the launch; its D_r^{-1/2}, residual and scratch rows are the b-th
  const int64_t sys = sys0 + blockIdx.x;
  const int64_t m = sys / K;
  const int k = (int)(sys % K);
  if (active && !active[m]) return;
  const int64_t Nx = (int64_t)n * n;
  const int64_t nx = (int64_t)n * (n + 1);
  const double* af = a + m * 2 * nx;
  const double* dr = dinvr + (int64_t)blockIdx.x * Nx;
  double2* q = (double2*)spec + sys * Nx;
  double2* res = (double2*)resbuf + (int64_t)blockIdx.x * Nx;
  float* base = scr + (int64_t)blockIdx.x * h.per_sys;
  float2* X = (float2*)base;
  float2* R = X + Nx;
  float2* P = R + Nx;
  float2* Q = P + Nx;
  double sv, cv;
  sincospi(-2.0 * k / N, &sv, &cv);
  const double an = exp(log(alpha) / N);
  const double lre = 1.0 - an * cv, lim = -an * sv;

  // level 0 operator, float64 residual, zero solution
  const MgLv<float2> v0 = mg_lv<float2>(base, h, 0);
  double bn[2] = {0.0, 0.0};
  const bool sm[2] = {false, true};
  for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
    const int i = (int)(p % n), j = (int)(p / n);
    v0.cw[p] = i >= 1 ? (float)(cT * af[(int64_t)j * (n + 1) + i] * dr[p - 1] * dr[p]) : 0.f;
    v0.cs[p] = j >= 1 ? (float)(cT * af[nx + (int64_t)j * n + i] * dr[p - n] * dr[p]) : 0.f;
    const float th = (float)(lim * dr[p] * dr[p]);
    v0.dg[p] = make_float2(1.f, th);
    const float den = 1.f + th * th;
    v0.di[p] = make_float2(1.f / den, -th / den);
    const double2 vv = q[p];
    res[p] = vv;
    q[p] = make_double2(0.0, 0.0);
    bn[0] += vv.x * vv.x + vv.y * vv.y;
    bn[1] = nanmax(bn[1], dr[p] * fmax(fabs(vv.x), fabs(vv.y)));
  }
  block_reduce<2>(bn, sm, dsl);   // its barriers also publish level 0
  mg_build_coarse<float2>(base, h);
  const double stop2 = rtol * rtol * bn[0];
  double rn2 = bn[0];
  double sig = bn[1];
  unsigned long long tot_it = 0, max_it = 0;
  int pass = 0;
  while (rn2 > stop2 && sig > 0.0 && pass < 12) {
    const double isig = 1.0 / sig;
    float r0 = 0.f;
    for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
      const double2 rv = res[p];
      const float2 vv = make_float2((float)(isig * dr[p] * rv.x), (float)(isig * dr[p] * rv.y));
      R[p] = vv;
      X[p] = make_float2(0.f, 0.f);
      r0 += vv.x * vv.x + vv.y * vv.y;
    }
    {
      float t[1] = {r0};
      block_sum_fk<NW, 1>(t, fsl[1], lane, wave);   // its barrier also publishes R
      r0 = t[0];
    }
    float2* Z = mg_vcycle<float2>(base, h, R);
    float acc2[2] = {0.f, 0.f};
    for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
      const float2 rv = R[p], zv = Z[p];
      P[p] = zv;
      acc2[0] += rv.x * zv.x - rv.y * zv.y;
      acc2[1] += rv.x * zv.y + rv.y * zv.x;
    }
    // one-barrier sums alternate between the two slot arrays: this one and the p.q sum
    // that follows with no barrier in between must not share slots
    block_sum_fk<NW, 2>(acc2, fsl[1], lane, wave);
    cf rz = {acc2[0], acc2[1]};
    float rr = r0;
    const float stop_in = inner_rtol * inner_rtol * r0;
    int it = 0;
    const int cap = maxit < 400 ? maxit : 400;
    bool bad = false;
    while (rr > stop_in && it < cap) {
      float pq2[2] = {0.f, 0.f};
      for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
        const int i = (int)(p % n), j = (int)(p / n);
        const float2 qv = mg_apply<float2>(v0, p, i, j, [&](int64_t s, int, int) { return P[s]; });
        Q[p] = qv;
        const float2 pv = P[p];
        pq2[0] += pv.x * qv.x - pv.y * qv.y;
        pq2[1] += pv.x * qv.y + pv.y * qv.x;
      }
      block_sum_fk<NW, 2>(pq2, fsl[0], lane, wave);
      const cf al = cf_div(rz, cf{pq2[0], pq2[1]});
      float racc[1] = {0.f};
      for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
        const float2 pv = P[p], qv = Q[p];
        float2 xv = X[p], rv = R[p];
        xv.x += al.x * pv.x - al.y * pv.y;
        xv.y += al.x * pv.y + al.y * pv.x;
        rv.x -= al.x * qv.x - al.y * qv.y;
        rv.y -= al.x * qv.y + al.y * qv.x;
        X[p] = xv;
        R[p] = rv;
        racc[0] += rv.x * rv.x + rv.y * rv.y;
      }
      block_sum_fk<NW, 1>(racc, fsl[1], lane, wave);   // its barrier also publishes R
      rr = racc[0];
      ++it;
      if (!(rr < 3.0e38f)) {
        bad = true;
        break;
      }
      if (rr <= stop_in) break;
      float rz2[2] = {0.f, 0.f};
      if (h.smoother == kMgGaussSeidel) {   // r.z accumulated by the V-cycle's last sweeps
        float2 d = make_float2(0.f, 0.f);
        Z = mg_vcycle_gs<float2>(base, h, R, &d);
        rz2[0] = d.x;
        rz2[1] = d.y;
      } else {
        Z = mg_vcycle<float2>(base, h, R);
        for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
          const float2 rv = R[p], zv = Z[p];
          rz2[0] += rv.x * zv.x - rv.y * zv.y;
          rz2[1] += rv.x * zv.y + rv.y * zv.x;
        }
      }
      block_sum_fk<NW, 2>(rz2, fsl[0], lane, wave);
      const cf rzn = {rz2[0], rz2[1]};
      const cf be = cf_div(rzn, rz);
      rz = rzn;
      if (!(fabsf(rz.x) + fabsf(rz.y) < 3.0e38f)) {
        bad = true;
        break;
      }
      for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
        const float2 pv = P[p], zv = Z[p];
        P[p] = make_float2(zv.x + be.x * pv.x - be.y * pv.y, zv.y + be.x * pv.y + be.y * pv.x);
      }
      __syncthreads();
    }
    tot_it += it;
    max_it = it > (int)max_it ? it : max_it;
    if (bad) {   // keep the last good q and report
      if (threadIdx.x == 0) atomicOr(flag, 1);
      break;
    }
    __syncthreads();   // X complete before neighbours are read below
    double acc[2] = {0.0, 0.0};
    for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
      const int i = (int)(p % n), j = (int)(p / n);
      const float2 xp = X[p];
      const double ex = sig * dr[p] * xp.x, ey = sig * dr[p] * xp.y;
      double sx = 0.0, sy = 0.0;
      const double aW = af[(int64_t)j * (n + 1) + i], aE = af[(int64_t)j * (n + 1) + i + 1];
      const double aS = af[nx + (int64_t)j * n + i], aN = af[nx + (int64_t)(j + 1) * n + i];
      double nxv = 0.0, nyv = 0.0;
      if (i > 0) { const float2 t = X[p - 1]; nxv = sig * dr[p - 1] * t.x; nyv = sig * dr[p - 1] * t.y; }
      sx += aW * (ex - nxv); sy += aW * (ey - nyv);
      nxv = nyv = 0.0;
      if (i < n - 1) { const float2 t = X[p + 1]; nxv = sig * dr[p + 1] * t.x; nyv = sig * dr[p + 1] * t.y; }
      sx += aE * (ex - nxv); sy += aE * (ey - nyv);
      nxv = nyv = 0.0;
      if (j > 0) { const float2 t = X[p - n]; nxv = sig * dr[p - n] * t.x; nyv = sig * dr[p - n] * t.y; }
      sx += aS * (ex - nxv); sy += aS * (ey - nyv);
      nxv = nyv = 0.0;
      if (j < n - 1) { const float2 t = X[p + n]; nxv = sig * dr[p + n] * t.x; nyv = sig * dr[p + n] * t.y; }
      sx += aN * (ex - nxv); sy += aN * (ey - nyv);
      const double mex = lre * ex - lim * ey + cT * sx;
      const double mey = lre * ey + lim * ex + cT * sy;
      double2 rv = res[p];
      rv.x -= mex;
      rv.y -= mey;
      res[p] = rv;
      double2 qv = q[p];
      qv.x += ex;
      qv.y += ey;
      q[p] = qv;
      acc[0] += rv.x * rv.x + rv.y * rv.y;
      acc[1] = nanmax(acc[1], dr[p] * fmax(fabs(rv.x), fabs(rv.y)));
    }
    block_reduce<2>(acc, sm, dsl);
    rn2 = acc[0];
    sig = acc[1];
    ++pass;
  }
  if (threadIdx.x == 0) {
    if (rn2 > stop2) {
      atomicOr(flag, 1);
      atomicAdd(&cnt[5], 1ull);
    }
    atomicAdd(&cnt[0], tot_it);
    atomicAdd(&cnt[1], (unsigned long long)pass);
    atomicAdd(&cnt[2], 1ull);
    atomicMax(&cnt[3], max_it);
  }
}

template <int NW, int CPL, int RPW>
void launch_cocg_resident(hipStream_t st, int64_t nsys, const double* a, const double* dr, int n, double cT,
                          int N, double alpha, double rtol, float inner_rtol, int maxit, const uint8_t* active,
                          double* spec, double* resbuf, int* flag, unsigned long long* cnt) {
  const size_t lds = sizeof(float2) * (size_t)n * n;
  // the attribute is set once per variant, to the largest tile it serves (n = 64 CPL RPW
  // / 8 columns by rows), before any launch that a graph capture could record
  static std::atomic<bool> attr_set{false};
  if (!attr_set.load()) {
    const int max_lds = (int)(sizeof(float2) * (size_t)(64 * CPL) * (size_t)(NW * RPW));
    KC_TRY_HIP(hipFuncSetAttribute((const void*)cocg_resident_kernel<NW, CPL, RPW>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, max_lds));
    attr_set.store(true);
  }
  cocg_resident_kernel<NW, CPL, RPW><<<dim3((unsigned)nsys), dim3(64 * NW), lds, st>>>(
      a, dr, n, cT, N, alpha, rtol, inner_rtol, maxit, active, spec, resbuf, flag, cnt);
  KC_LAUNCH_CHECK();
}

template <int C>
size_t fft_lds(int N) {
  return sizeof(cd) * ((size_t)N * C + N / 2);
}

}  // namespace

void launch_defect(hipStream_t s, const klecgc_problem& p, const double* a, const double* Fv,
                   const double* U, const uint8_t* active, int64_t M, double* D) {
  const int64_t Nx = n_unknowns(p);
  const double h = 1.0 / (p.n + 1);
  const double cT = (p.T / p.N) / (h * h);
  dim3 grid((unsigned)((Nx + 255) / 256), (unsigned)(M * p.N));
  defect_kernel<<<grid, dim3(256), 0, s>>>(a, p.dim, p.n, cT, Fv, U, active, M, p.N, D);
  KC_LAUNCH_CHECK();
}

static int ilog2(int N) {
  int l = 0;
  while ((1 << l) < N) ++l;
  return l;
}

// Columns per work-group C and threads per column T (C T = 256): the [N][C] complex LDS
// tile stays at 32 KB for N >= 32; for N <= 4 the columns take one thread each.
#define KC_FFT_LAUNCH(KERNEL, C_, T_, ...)                                                      \
  KERNEL<C_, T_><<<dim3((unsigned)((Nx_ + (C_) - 1) / (C_)), (unsigned)M), dim3((C_) * (T_)), fft_lds<C_>(p.N), s>>>( \
      __VA_ARGS__)
#define KC_FFT_DISPATCH(KERNEL, ...)                                                            \
  do {                                                                                          \
    const int64_t Nx_ = n_unknowns(p);                                                          \
    if (p.N <= 4)                                                                               \
      KC_FFT_LAUNCH(KERNEL, 256, 1, __VA_ARGS__);                                               \
    else if (p.N <= 32)                                                                         \
      KC_FFT_LAUNCH(KERNEL, 64, 4, __VA_ARGS__);                                                \
    else if (p.N == 64)                                                                         \
      KC_FFT_LAUNCH(KERNEL, 32, 8, __VA_ARGS__);                                                \
    else if (p.N == 128)                                                                        \
      KC_FFT_LAUNCH(KERNEL, 16, 16, __VA_ARGS__);                                               \
    else                                                                                        \
      KC_FFT_LAUNCH(KERNEL, 8, 32, __VA_ARGS__);                                                \
    KC_LAUNCH_CHECK();                                                                          \
  } while (0)

void launch_fft_forward(hipStream_t s, const klecgc_problem& p, const double* r,
                        const uint8_t* active, int64_t M, double* spec) {
  const int64_t Nx = n_unknowns(p);
  const int logn = ilog2(p.N);
  KC_FFT_DISPATCH(fft_forward_kernel, r, Nx, p.N, logn, p.alpha, active, spec);
}

void launch_fft_inverse(hipStream_t s, const klecgc_problem& p, const double* spec,
                        const uint8_t* active, int64_t M, double* u, bool accumulate,
                        unsigned long long* maxima) {
  const int64_t Nx = n_unknowns(p);
  const int logn = ilog2(p.N);
  KC_FFT_DISPATCH(fft_inverse_kernel, spec, Nx, p.N, logn, p.alpha, active, u, accumulate ? 1 : 0, maxima);
}

int shifted_solve_impl(klecgc_ctx* ctx, const klecgc_problem& p, const double* a,
                       const uint8_t* active, int64_t M, double* spec) {
  hipStream_t st = ctx->stream;
  const int K = p.N / 2 + 1;
  const int64_t Nx = n_unknowns(p);
  const double h = 1.0 / (p.n + 1);
  const double cT = (p.T / p.N) / (h * h);
  const int64_t nsys = M * K;
  if (p.dim == 1) {
    double* scr = (double*)ctx->ws.get(WS_FACTORS, sizeof(double) * 2 * Nx * nsys);
    timed(ctx, KT_SHIFTED, [&] {
      shifted_tri_kernel<<<dim3((unsigned)((nsys + 63) / 64)), dim3(64), 0, st>>>(
          a, p.n, cT, p.N, p.alpha, active, M, spec, scr);
      KC_LAUNCH_CHECK();
    });
    return KC_OK;
  }
  DevStatus ds = status_block(ctx, WS_STATUS_CGC);
  status_reset(ctx, ds);
  const double rtol = p.cgc_rtol > 0 ? p.cgc_rtol : 1e-13;
  const int maxit = p.cgc_max_iter > 0 ? p.cgc_max_iter : 20000;
  const KcTuning tu = tuning_for(ctx, p.n);
  const int variant = p.precision == KC_PREC_F32_REFINED ? cgc_variant_for(p.n, tu.cgc_variant) : KC_CGC_STREAM64;
  const float inner = tu.cgc_inner_rtol;
  if (variant == KC_CGC_MG32) {
    const MgLevels h = mg_levels(p.n, 2, 8LL * Nx, tu.mg_sweeps, tu.mg_smoother);
    // systems run in chunks whose D_r^{-1/2}, residuals and scratch take at most 16 GiB
    const int64_t per_sys = (int64_t)sizeof(double) * 3 * Nx + (int64_t)sizeof(float) * h.per_sys;
    const int64_t chunk = std::min<int64_t>(nsys, std::max<int64_t>(4LL * ctx->num_cus, ((int64_t)16 << 30) / per_sys));
    double* dr = (double*)ctx->ws.get(WS_DINV, sizeof(double) * Nx * chunk);
    double* resb = (double*)ctx->ws.get(WS_KRYLOV, sizeof(double) * 2 * Nx * chunk);
    float* scr = (float*)ctx->ws.get(WS_FINE_AUX, sizeof(float) * h.per_sys * chunk);
    timed(ctx, KT_SHIFTED, [&] {
      for (int64_t s0 = 0; s0 < nsys; s0 += chunk) {
        const int64_t cs = std::min<int64_t>(chunk, nsys - s0);
        shift_dinv_kernel<<<dim3((unsigned)((Nx + 255) / 256), (unsigned)cs), dim3(256), 0, st>>>(
            a, p.n, cT, p.N, p.alpha, M, dr, s0);
        KC_LAUNCH_CHECK();
        // 16 waves per system, one work-group per CU: the node loops are latency-bound and
        // gain most from the waves one system can keep in flight
        cocg_mg_kernel<16, 4><<<dim3((unsigned)cs), dim3(1024), 0, st>>>(
            a, dr, p.n, cT, p.N, p.alpha, rtol, inner, maxit, active, spec, resb, scr, h, ds.flag, ds.cnt, s0);
        KC_LAUNCH_CHECK();
      }
    });
    return status_collect(ctx, ds, 4) ? KC_ENOCONV : KC_OK;
  }
  if (variant == KC_CGC_STREAM32) {
    double* dr = (double*)ctx->ws.get(WS_DINV, sizeof(double) * Nx * nsys);
    double* resb = (double*)ctx->ws.get(WS_KRYLOV, sizeof(double) * 2 * Nx * nsys);
    float* scr = (float*)ctx->ws.get(WS_FINE_AUX, sizeof(float) * 11 * Nx * nsys);
    shift_dinv_kernel<<<dim3((unsigned)((Nx + 255) / 256), (unsigned)nsys), dim3(256), 0, st>>>(
        a, p.n, cT, p.N, p.alpha, M, dr);
    KC_LAUNCH_CHECK();
    timed(ctx, KT_SHIFTED, [&] {
      cocg32_stream_kernel<<<dim3((unsigned)nsys), dim3(512), 0, st>>>(
          a, dr, p.n, cT, p.N, p.alpha, rtol, inner, maxit, active, spec, resb, scr, ds.flag, ds.cnt);
      KC_LAUNCH_CHECK();
    });
    return status_collect(ctx, ds, 4) ? KC_ENOCONV : KC_OK;
  }
  if (variant != KC_CGC_STREAM64) {
    double* dr = (double*)ctx->ws.get(WS_DINV, sizeof(double) * Nx * nsys);
    double* resb = (double*)ctx->ws.get(WS_KRYLOV, sizeof(double) * 2 * Nx * nsys);
    shift_dinv_kernel<<<dim3((unsigned)((Nx + 255) / 256), (unsigned)nsys), dim3(256), 0, st>>>(
        a, p.n, cT, p.N, p.alpha, M, dr);
    KC_LAUNCH_CHECK();
    timed(ctx, KT_SHIFTED, [&] {
      // 8 waves; one grid row block of RPW rows per wave, one column per lane
      if (variant == KC_CGC_RES16)
        launch_cocg_resident<8, 1, 2>(st, nsys, a, dr, p.n, cT, p.N, p.alpha, rtol, inner, maxit, active, spec,
                                      resb, ds.flag, ds.cnt);
      else if (variant == KC_CGC_RES32)
        launch_cocg_resident<8, 1, 4>(st, nsys, a, dr, p.n, cT, p.N, p.alpha, rtol, inner, maxit, active, spec,
                                      resb, ds.flag, ds.cnt);
      else
        launch_cocg_resident<8, 1, 8>(st, nsys, a, dr, p.n, cT, p.N, p.alpha, rtol, inner, maxit, active, spec,
                                      resb, ds.flag, ds.cnt);
    });
    return status_collect(ctx, ds, 4) ? KC_ENOCONV : KC_OK;
  }
  double* scr = (double*)ctx->ws.get(WS_KRYLOV, sizeof(double) * 6 * Nx * nsys);
  timed(ctx, KT_SHIFTED, [&] {
    cocg_kernel<<<dim3((unsigned)nsys), dim3(kCocgThreads), 0, st>>>(a, p.n, cT, p.N, p.alpha, rtol,
                                                                     maxit, active, spec, scr, ds.flag, ds.cnt);
    KC_LAUNCH_CHECK();
  });
  return status_collect(ctx, ds, 4) ? KC_ENOCONV : KC_OK;
}

bool cgc_variant_fits(int v, int n) {
  switch (v) {
    case KC_CGC_STREAM64: return true;
    case KC_CGC_RES16: return n <= 16;
    case KC_CGC_RES32: return n <= 32;
    case KC_CGC_RES64: return n <= 64;
    case KC_CGC_STREAM32: return true;
    case KC_CGC_MG32: return true;
    default: return false;
  }
}

int cgc_variant_for(int n, int requested) {
  if (requested >= 0 && cgc_variant_fits(requested, n)) return requested;
  if (n <= 16) return KC_CGC_RES16;
  if (n <= 32) return KC_CGC_RES32;
  if (n <= 64) return KC_CGC_RES64;
  return KC_CGC_MG32;
}

}  // namespace kc
