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

#include "common.h"
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
// One thread per column (m, x); COLS consecutive x per work-group; the column's N
// values live in LDS as [N][COLS] complex so that a wave touches contiguous words.
template <int COLS>
__device__ void fft_inplace(cd* buf, const cd* tw, int N, int logn, int t) {
  for (int len = 2; len <= N; len <<= 1) {
    const int half = len >> 1;
    const int stride = N / len;
    for (int start = 0; start < N; start += len) {
      for (int k = 0; k < half; ++k) {
        cd w = tw[k * stride];
        cd u = buf[(start + k) * COLS + t];
        cd v = buf[(start + k + half) * COLS + t] * w;
        buf[(start + k) * COLS + t] = u + v;
        buf[(start + k + half) * COLS + t] = u - v;
      }
    }
  }
}

template <int COLS>
__global__ __launch_bounds__(COLS) void fft_forward_kernel(const double* __restrict__ r, int64_t Nx,
                                                           int N, int logn, double alpha,
                                                           const uint8_t* __restrict__ active,
                                                           double* __restrict__ spec) {
  extern __shared__ cd lds[];
  cd* buf = lds;                 // [N][COLS]
  cd* tw = lds + N * COLS;       // [N/2] e^{-2 pi i k / N}
  const int t = threadIdx.x;
  const int64_t m = blockIdx.y;
  if (active && !active[m]) return;
  for (int k = t; k < N / 2; k += COLS) {
    double sv, cv;
    sincospi(-2.0 * k / N, &sv, &cv);
    tw[k] = {cv, sv};
  }
  const int64_t x = (int64_t)blockIdx.x * COLS + t;
  const double invsq = 1.0 / sqrt((double)N);
  const double la = log(alpha) / N;
  if (x < Nx) {
    const double* col = r + m * N * Nx + x;
    for (int s = 0; s < N; ++s) {
      double sc = exp(la * s);   // alpha^{s/N}
      buf[bitrev(s, logn) * COLS + t] = {sc * col[(int64_t)s * Nx], 0.0};
    }
  }
  __syncthreads();
  if (x < Nx) {
    fft_inplace<COLS>(buf, tw, N, logn, t);
    const int K = N / 2 + 1;
    cd* out = (cd*)spec + m * K * Nx + x;
    for (int k = 0; k < K; ++k) out[(int64_t)k * Nx] = invsq * buf[k * COLS + t];
  }
}

// u_s = alpha^{-s/N} Re( N^{-1/2} sum_k e^{+2 pi i k s/N} Q_k ), Q_{N-k} = conj(Q_k).
// accumulate: u += result; maxima[m] = {max |result|, max |u_new|} as ordered bit patterns.
template <int COLS>
__global__ __launch_bounds__(COLS) void fft_inverse_kernel(const double* __restrict__ spec,
                                                           int64_t Nx, int N, int logn,
                                                           double alpha,
                                                           const uint8_t* __restrict__ active,
                                                           double* __restrict__ u, int accumulate,
                                                           unsigned long long* __restrict__ maxima) {
  extern __shared__ cd lds[];
  cd* buf = lds;
  cd* tw = lds + N * COLS;       // e^{+2 pi i k / N}
  const int t = threadIdx.x;
  const int64_t m = blockIdx.y;
  if (active && !active[m]) return;
  for (int k = t; k < N / 2; k += COLS) {
    double sv, cv;
    sincospi(2.0 * k / N, &sv, &cv);
    tw[k] = {cv, sv};
  }
  const int64_t x = (int64_t)blockIdx.x * COLS + t;
  const int K = N / 2 + 1;
  if (x < Nx) {
    const cd* in = (const cd*)spec + m * K * Nx + x;
    for (int k = 0; k < K; ++k) {
      cd q = in[(int64_t)k * Nx];
      buf[bitrev(k, logn) * COLS + t] = q;
      if (k > 0 && k < N - k) buf[bitrev(N - k, logn) * COLS + t] = conj(q);
    }
  }
  __syncthreads();
  double cmax = 0.0, umax = 0.0;
  if (x < Nx) {
    fft_inplace<COLS>(buf, tw, N, logn, t);
    const double invsq = 1.0 / sqrt((double)N);
    const double la = -log(alpha) / N;
    double* col = u + m * N * Nx + x;
    for (int s = 0; s < N; ++s) {
      double v = exp(la * s) * invsq * buf[s * COLS + t].x;
      double* dst = col + (int64_t)s * Nx;
      if (accumulate) {
        double nu = *dst + v;
        *dst = nu;
        cmax = nanmax(cmax, fabs(v));
        umax = nanmax(umax, fabs(nu));
      } else {
        *dst = v;
      }
    }
  }
  if (maxima) {
    // non-negative doubles order like their bit patterns
    if (COLS >= 64) {
      cmax = wave_nanmax(cmax);
      umax = wave_nanmax(umax);
    }
    if (COLS < 64 || (t & 63) == 0) {
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

template <int COLS>
size_t fft_lds(int N) {
  return sizeof(cd) * ((size_t)N * COLS + N / 2);
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

// Columns per work-group: the [N][COLS] complex LDS tile stays at 32 KB (N >= 32).
#define KC_FFT_DISPATCH(KERNEL, ...)                                                            \
  do {                                                                                          \
    const int64_t Nx_ = n_unknowns(p);                                                          \
    if (p.N <= 32) {                                                                            \
      constexpr int C = 64;                                                                     \
      KERNEL<C><<<dim3((unsigned)((Nx_ + C - 1) / C), (unsigned)M), dim3(C), fft_lds<C>(p.N), s>>>(__VA_ARGS__); \
    } else if (p.N == 64) {                                                                     \
      constexpr int C = 32;                                                                     \
      KERNEL<C><<<dim3((unsigned)((Nx_ + C - 1) / C), (unsigned)M), dim3(C), fft_lds<C>(p.N), s>>>(__VA_ARGS__); \
    } else if (p.N == 128) {                                                                    \
      constexpr int C = 16;                                                                     \
      KERNEL<C><<<dim3((unsigned)((Nx_ + C - 1) / C), (unsigned)M), dim3(C), fft_lds<C>(p.N), s>>>(__VA_ARGS__); \
    } else {                                                                                    \
      constexpr int C = 8;                                                                      \
      KERNEL<C><<<dim3((unsigned)((Nx_ + C - 1) / C), (unsigned)M), dim3(C), fft_lds<C>(p.N), s>>>(__VA_ARGS__); \
    }                                                                                           \
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
    shifted_tri_kernel<<<dim3((unsigned)((nsys + 63) / 64)), dim3(64), 0, st>>>(
        a, p.n, cT, p.N, p.alpha, active, M, spec, scr);
    KC_LAUNCH_CHECK();
    return KC_OK;
  }
  double* scr = (double*)ctx->ws.get(WS_KRYLOV, sizeof(double) * 6 * Nx * nsys);
  DevStatus ds = status_block(ctx);
  status_reset(ctx, ds);
  const double rtol = p.cgc_rtol > 0 ? p.cgc_rtol : 1e-13;
  const int maxit = p.cgc_max_iter > 0 ? p.cgc_max_iter : 20000;
  cocg_kernel<<<dim3((unsigned)nsys), dim3(kCocgThreads), 0, st>>>(a, p.n, cT, p.N, p.alpha, rtol,
                                                                   maxit, active, spec, scr, ds.flag, ds.cnt);
  KC_LAUNCH_CHECK();
  return status_collect(ctx, ds, 4) ? KC_ENOCONV : KC_OK;
}

}  // namespace kc
