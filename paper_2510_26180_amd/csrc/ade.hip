// The advection-diffusion example of Section 5.1 on the GPU: P1 finite elements on the
// uniform n x n interior grid (each cell cut by its rising diagonal), backward Euler for F
// and G, and the diagonalised coarse grid correction with the mass matrix,
//     (C_alpha (x) M + dT I (x) L) u = r,  L = a K + B                       (Section 3.2)
// solved as N/2+1 shifted systems (lambda_k M + dT L) q_k = p_k.
//
// The systems are small (n <= 31, natural ordering, half-bandwidth n+1 <= 32) and the same
// matrix serves every step of a sample, so everything is a direct banded solve:
//   * band LU without pivoting, one 64-thread work-group per matrix, rows assembled from the
//     element stencils into a circular LDS window of W+1 rows as the elimination advances
//     (the symmetric part of every matrix here, Re(lambda) M + tau a K, is positive definite
//     because the advection matrix is skew for div b = 0, so no pivot vanishes);
//   * the fine sweep: one wavefront per sample, lane = slice, the sample's factor read with
//     wave-uniform (scalar) loads, the W-row window of the substitutions held in registers
//     (W a template parameter, fully unrolled), the state of each lane in a [Nx][64]
//     column of device memory (coalesced across the lanes);
//   * the shifted solves of step (b): one wavefront per (sample, bin), factor rows staged
//     through LDS 32 at a time, the substitution window across lanes 0..W-1 and a
//     32-lane reduction per row.
#include <cmath>
#include <vector>

#include "models.h"
#include "reduce.h"

namespace kc {

namespace {

constexpr int kTab = 32;      // per-node table: M[7], K[7], B[7], l0, l1, M[7] with the couplings to
                              // boundary nodes zeroed, (pad)
constexpr int kMaxW = 32;     // largest half-bandwidth (n <= 31)
constexpr int kStage = 32;    // factor rows staged per LDS chunk in the shifted solves
// slices per wavefront in the fine sweep: each wavefront stages its sample's factor twice per
// step and makes six passes over its lane states, so dealing a sample's slices to several
// wavefronts multiplies that traffic (8 slices per wavefront measured 2.8x slower than 64)
constexpr int kSweepLanes = 64;

// stencil slot s -> neighbour offset (di, dj): 0 centre, 1 (-1,0), 2 (+1,0), 3 (0,-1),
// 4 (0,+1), 5 (+1,+1), 6 (-1,-1) (the P1 couplings on this mesh)
__host__ __device__ __forceinline__ int slot_di(int s) {
  return s == 1 ? -1 : (s == 2 || s == 5) ? 1 : s == 6 ? -1 : 0;
}
__host__ __device__ __forceinline__ int slot_dj(int s) {
  return s == 3 ? -1 : (s == 4 || s == 5) ? 1 : s == 6 ? -1 : 0;
}
__device__ __forceinline__ int slot_of(int di, int dj) {
  for (int s = 0; s < 7; ++s)
    if (slot_di(s) == di && slot_dj(s) == dj) return s;
  return -1;
}

__device__ __forceinline__ cplx operator*(cplx a, cplx b) {
  return cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx operator-(cplx a, cplx b) { return cplx{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx recip(cplx a) {
  const double d = a.re * a.re + a.im * a.im;
  return cplx{a.re / d, -a.im / d};
}
__device__ __forceinline__ double recip(double a) { return 1.0 / a; }
__device__ __forceinline__ bool usable_pivot(double a) { return isfinite(a) && a != 0.0; }
__device__ __forceinline__ bool usable_pivot(cplx a) {
  return isfinite(a.re) && isfinite(a.im) && (a.re != 0.0 || a.im != 0.0);
}
template <class T> __device__ __forceinline__ T zero_of();
template <> __device__ __forceinline__ double zero_of<double>() { return 0.0; }
template <> __device__ __forceinline__ cplx zero_of<cplx>() { return cplx{0.0, 0.0}; }
// sigma M + lv with the real (sre) or complex (sre + i sim) shift sigma
template <class T> __device__ __forceinline__ T band_value(double sre, double sim, double mv, double lv);
template <> __device__ __forceinline__ double band_value<double>(double sre, double, double mv, double lv) {
  return sre * mv + lv;
}
template <> __device__ __forceinline__ cplx band_value<cplx>(double sre, double sim, double mv, double lv) {
  return cplx{sre * mv + lv, sim * mv};
}

// the source of Section 5.1, f = exp(-t) (g0 + a g1)
__device__ __forceinline__ double src_g0(double x1, double x2, double beta) {
  const double s1 = sinpi(x1), s2 = sinpi(2.0 * x2);
  return -s1 * s2 + 0.5 * beta * M_PI * x2 * cospi(x1) * s2 + beta * M_PI * x1 * s1 * cospi(2.0 * x2);
}
__device__ __forceinline__ double src_g1(double x1, double x2) { return M_PI * M_PI * sinpi(x1) * sinpi(2.0 * x2); }

// Element-by-element stencils of interior node p = (i, j): the six triangles around it,
// exact P1 integrals (area h^2/2, constant gradients, b linear so that
// int_T b phi_a = |T|/12 (sum_k b(x_k) + b(x_a))), and the load pieces l0, l1 = the mass
// stencil applied to g0, g1 at the seven grid nodes (boundary nodes included).
__global__ void ade_tables_kernel(int n, double beta, double* __restrict__ tab) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n * n) return;
  const int gi = p % n + 1, gj = p / n + 1;
  const double h = 1.0 / (n + 1);
  const double area = 0.5 * h * h;
  double Mv[7], Kv[7], Bv[7];
  for (int s = 0; s < 7; ++s) Mv[s] = Kv[s] = Bv[s] = 0.0;
  for (int cell = 0; cell < 4; ++cell) {
    const int ci = gi - 1 + (cell & 1), cj = gj - 1 + (cell >> 1);
    for (int tri = 0; tri < 2; ++tri) {
      int vi[3], vj[3];
      vi[0] = ci;
      vj[0] = cj;
      vi[1] = ci + 1;
      vj[1] = tri == 0 ? cj : cj + 1;
      vi[2] = tri == 0 ? ci + 1 : ci;
      vj[2] = cj + 1;
      int a = -1;
      for (int k = 0; k < 3; ++k)
        if (vi[k] == gi && vj[k] == gj) a = k;
      if (a < 0) continue;
      double x[3], y[3], gx[3], gy[3];
      for (int k = 0; k < 3; ++k) {
        x[k] = vi[k] * h;
        y[k] = vj[k] * h;
      }
      for (int k = 0; k < 3; ++k) {
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        gx[k] = (y[k1] - y[k2]) / (2.0 * area);
        gy[k] = (x[k2] - x[k1]) / (2.0 * area);
      }
      const double sbx = beta * (y[0] + y[1] + y[2] + y[a]);
      const double sby = beta * (x[0] + x[1] + x[2] + x[a]);
      for (int c = 0; c < 3; ++c) {
        const int s = slot_of(vi[c] - gi, vj[c] - gj);
        Mv[s] += area * (c == a ? 2.0 : 1.0) / 12.0;
        Kv[s] += area * (gx[a] * gx[c] + gy[a] * gy[c]);
        Bv[s] += area / 12.0 * (sbx * gx[c] + sby * gy[c]);
      }
    }
  }
  double l0 = 0.0, l1 = 0.0;
  for (int s = 0; s < 7; ++s) {
    const double x1 = (gi + slot_di(s)) * h, x2 = (gj + slot_dj(s)) * h;
    l0 += Mv[s] * src_g0(x1, x2, beta);
    l1 += Mv[s] * src_g1(x1, x2);
  }
  double* t = tab + (size_t)p * kTab;
  for (int s = 0; s < 7; ++s) {
    t[s] = Mv[s];
    t[7 + s] = Kv[s];
    t[14 + s] = Bv[s];
  }
  t[21] = l0;
  t[22] = l1;
  for (int s = 0; s < 7; ++s) {
    const int ii = gi + slot_di(s), jj = gj + slot_dj(s);
    t[23 + s] = (ii >= 1 && ii <= n && jj >= 1 && jj <= n) ? Mv[s] : 0.0;
  }
  t[30] = t[31] = 0.0;
}

__global__ void ade_u0_kernel(int n, int64_t M, double* __restrict__ u0) {
  const int64_t Nx = (int64_t)n * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < M * Nx; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = t % Nx;
    const double h = 1.0 / (n + 1);
    const double x1 = (double)(p % n + 1) * h, x2 = (double)(p / n + 1) * h;
    u0[t] = sinpi(x1) * sinpi(2.0 * x2);
  }
}

// Row p of sigma M + tau (a K + B) in band form (entry e <-> column p - W + e), filled by the
// work-group's threads; couplings to boundary nodes are dropped (zero Dirichlet data).
template <class T>
__device__ void assemble_row(const double* __restrict__ tab, int n, int W, int p, double a, double tau, double sre,
                             double sim, T* row) {
  const int i = p % n, j = p / n;
  const double* t = tab + (size_t)p * kTab;
  for (int e = threadIdx.x; e < 2 * W + 1; e += blockDim.x) {
    const int off = e - W;
    T v = zero_of<T>();
    for (int s = 0; s < 7; ++s) {
      const int di = slot_di(s), dj = slot_dj(s);
      if (di + n * dj == off && i + di >= 0 && i + di < n && j + dj >= 0 && j + dj < n)
        v = band_value<T>(sre, sim, t[s], tau * (a * t[7 + s] + t[14 + s]));
    }
    row[e] = v;
  }
}

// Band LU (no pivoting) of sys = (sample m, bin k): sigma M + tau (a_m K + B), sigma = 1 (real
// factors) or lambda_k = 1 - alpha^{1/N} e^{-2 pi i k / N} (complex).  Output row p of
// fac[sys] ([Nx][2W+1]): entries e < W the multipliers L[p][p-W+e], e = W the reciprocal of
// U[p][p], e > W the entries U[p][p-W+e].  bad[sys] = 1 on an unusable pivot.
template <class T>
__global__ __launch_bounds__(64) void ade_factor_kernel(const double* __restrict__ tab, int n, int W,
                                                        const double* __restrict__ coef, int K, int N, double aroot,
                                                        double tau, int complex_shift, T* __restrict__ fac,
                                                        int* __restrict__ bad) {
  extern __shared__ unsigned char smem[];
  T* rows = reinterpret_cast<T*>(smem);        // [W+1][2W+1] circular window
  T* lbuf = rows + (W + 1) * (2 * W + 1);      // [W] multipliers of the current pivot
  const int64_t sys = blockIdx.x;
  const int64_t m = sys / K;
  const int k = (int)(sys % K);
  const int Nx = n * n, BW = 2 * W + 1;
  double sre = 1.0, sim = 0.0;
  if (complex_shift) {
    const double th = 2.0 * M_PI * (double)k / (double)N;
    sre = 1.0 - aroot * cos(th);
    sim = aroot * sin(th);
  }
  const double a = coef[m];
  T* out = fac + (size_t)sys * Nx * BW;
  for (int r = 0; r <= W && r < Nx; ++r) assemble_row<T>(tab, n, W, r, a, tau, sre, sim, rows + (r % (W + 1)) * BW);
  int isbad = 0;
  for (int p = 0; p < Nx; ++p) {
    __syncthreads();
    T* rp = rows + (p % (W + 1)) * BW;
    const T piv = rp[W];
    if (!usable_pivot(piv)) isbad = 1;
    const T ipiv = recip(piv);
    if ((int)threadIdx.x < W) {
      const int rr = threadIdx.x + 1;
      lbuf[threadIdx.x] = (p + rr < Nx) ? rows[((p + rr) % (W + 1)) * BW + W - rr] * ipiv : zero_of<T>();
    }
    __syncthreads();
    for (int q = threadIdx.x; q < W * W; q += blockDim.x) {
      const int rr = q / W + 1, cc = q % W + 1;
      if (p + rr < Nx && p + cc < Nx) {
        T* rowr = rows + ((p + rr) % (W + 1)) * BW;
        rowr[W - rr + cc] = rowr[W - rr + cc] - lbuf[rr - 1] * rp[W + cc];
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < W) {
      const int rr = threadIdx.x + 1;
      if (p + rr < Nx) rows[((p + rr) % (W + 1)) * BW + W - rr] = lbuf[threadIdx.x];
    }
    for (int e = threadIdx.x; e < BW; e += blockDim.x) out[(size_t)p * BW + e] = (e == W) ? ipiv : rp[e];
    __syncthreads();
    if (p + W + 1 < Nx) assemble_row<T>(tab, n, W, p + W + 1, a, tau, sre, sim, rp);
  }
  if (threadIdx.x == 0 && isbad) bad[sys] = 1;
}

// One wavefront per listed sample, lane l <-> slice s_lo + l (l < nsl).  J backward-Euler steps
// of size tau; step j of slice s ends at t = s dT + (j+1) tau:
//   (M + tau L) w' = M w + tau exp(-t) (l0 + a l1)
// by the sample's band LU.  work: [nlist][2][Nx + 2(n+1)][64]: w between n+1 zero ghost rows on
// either side, then the right-hand side / forward-substituted y.  Each step: (1) the right-hand
// sides of all rows, branch-free (the ghost rows and the interior-masked mass couplings stand in
// for the boundary), so the loads of consecutive rows overlap; (2) forward and (3) back
// substitution in blocks of W rows: the factor rows of
// the next block are loaded (coalesced over the lanes) while the current block computes from
// LDS, and the next block's right-hand sides are loaded into registers the same way, so a row
// waits only on LDS and its own recurrence.
template <int W>
__global__ __launch_bounds__(64) void ade_sweep_kernel(const double* __restrict__ tab, int n,
                                                       const double* __restrict__ coef,
                                                       const double* __restrict__ fac,
                                                       const int32_t* __restrict__ list, const double* __restrict__ base,
                                                       const double* __restrict__ u0, int shift, int s_lo, int nsl,
                                                       int lanes, int N, int J, double tau, double dT,
                                                       double* __restrict__ work, double* __restrict__ out) {
  constexpr int BW = 2 * W + 1;
  constexpr int BLK = W * BW;              // factor entries of one block of W rows
  constexpr int SR = (BLK + 63) / 64;      // staged entries per lane
  __shared__ double stg[2][BLK];
  // the sample's slices are dealt to ceil(nsl / lanes) wavefronts, `lanes` slices each
  const int waves = (nsl + lanes - 1) / lanes;
  const int li = blockIdx.x / waves;
  const int part = blockIdx.x % waves;
  const int64_t m = list ? list[li] : li;
  const int lane = threadIdx.x;
  const bool on = lane < lanes && part * lanes + lane < nsl;
  const int s = s_lo + part * lanes + lane;
  const int Nx = n * n;
  const int G = n + 1;                       // ghost rows on either side of w
  const double* F = fac + (size_t)m * Nx * BW;
  double* wg = work + (size_t)blockIdx.x * 2 * (Nx + 2 * G) * 64 + lane;
  double* w = wg + (size_t)G * 64;
  double* y = wg + (size_t)(Nx + 2 * G) * 64;
  const double a = coef[m];
  const double* src = nullptr;
  if (on)
    src = shift ? (s == 0 ? u0 + m * Nx : base + (m * N + s - 1) * Nx) : base + (m * N + s) * Nx;
  for (int p = 0; p < G; ++p) {
    wg[(size_t)p * 64] = 0.0;
    w[(size_t)(Nx + p) * 64] = 0.0;
  }
#pragma unroll 4
  for (int p = 0; p < Nx; ++p) w[(size_t)p * 64] = on ? src[p] : 0.0;
  const double t0 = (double)s * dT;
  const int64_t off[7] = {0, -64, 64, -(int64_t)n * 64, (int64_t)n * 64, (int64_t)(n + 1) * 64,
                          -(int64_t)(n + 1) * 64};
  // factor rows [rlo, rlo + W) of the sample (rows outside [0, Nx) read as 0)
  auto stage_load = [&](int rlo, double (&reg)[SR]) {
#pragma unroll
    for (int q = 0; q < SR; ++q) {
      const int e = lane + 64 * q;
      const int row = rlo + e / BW;
      reg[q] = (e < BLK && row >= 0 && row < Nx) ? F[(int64_t)rlo * BW + e] : 0.0;
    }
  };
  auto stage_store = [&](double* buf, const double (&reg)[SR]) {
#pragma unroll
    for (int q = 0; q < SR; ++q) {
      const int e = lane + 64 * q;
      if (e < BLK) buf[e] = reg[q];
    }
  };
  double win[W], rc[W], rn[W], sreg[SR];
#pragma unroll
  for (int r = 0; r < W; ++r) win[r] = 0.0;
  const int nblk = (Nx + W - 1) / W;
  for (int j = 0; j < J; ++j) {
    const double et = tau * exp(-(t0 + (double)(j + 1) * tau));
    // (1) right-hand sides M w + tau F(t) into y
#pragma unroll 8
    for (int p = 0; p < Nx; ++p) {
      const double* t = tab + (size_t)p * kTab;
      const double* wp = w + (size_t)p * 64;
      double acc = t[23] * wp[off[0]];
#pragma unroll
      for (int q = 1; q < 7; ++q) acc += t[23 + q] * wp[off[q]];
      y[(size_t)p * 64] = acc + et * (t[21] + a * t[22]);
    }
    // (2) forward substitution, blocks of rows [bW, bW + W)
#pragma unroll
    for (int r = 0; r < W; ++r) win[r] = 0.0;
    stage_load(0, sreg);
#pragma unroll
    for (int r = 0; r < W; ++r) rc[r] = r < Nx ? y[(size_t)r * 64] : 0.0;
    __syncthreads();
    stage_store(stg[0], sreg);
    __syncthreads();
    for (int b = 0; b < nblk; ++b) {
      const int p0 = b * W;
      const bool more = b + 1 < nblk;
      if (more) {
        stage_load(p0 + W, sreg);
#pragma unroll
        for (int r = 0; r < W; ++r) rn[r] = (p0 + W + r < Nx) ? y[(size_t)(p0 + W + r) * 64] : 0.0;
      }
      const double* S = stg[b & 1];
#pragma unroll
      for (int r = 0; r < W; ++r) {
        const int p = p0 + r;
        if (p < Nx) {
          // band entries of columns below 0 are zero, and so is the window before row 0
          double acc = rc[r], acc2 = 0.0;
#pragma unroll
          for (int k = 1; k <= W; ++k) {
            if (k & 1)
              acc -= S[r * BW + W - k] * win[(r - k + W) % W];
            else
              acc2 -= S[r * BW + W - k] * win[(r - k + W) % W];
          }
          acc += acc2;
          win[r] = acc;
          y[(size_t)p * 64] = acc;
        }
      }
      if (more) {
        stage_store(stg[(b + 1) & 1], sreg);
#pragma unroll
        for (int r = 0; r < W; ++r) rc[r] = rn[r];
      }
      __syncthreads();
    }
    // (3) back substitution, blocks of rows (p0 - W, p0], p0 = Nx - 1 - bW
#pragma unroll
    for (int r = 0; r < W; ++r) win[r] = 0.0;
    stage_load(Nx - W, sreg);
#pragma unroll
    for (int r = 0; r < W; ++r) rc[r] = (Nx - 1 - r >= 0) ? y[(size_t)(Nx - 1 - r) * 64] : 0.0;
    stage_store(stg[0], sreg);
    __syncthreads();
    for (int b = 0; b < nblk; ++b) {
      const int p0 = Nx - 1 - b * W;
      const bool more = b + 1 < nblk;
      if (more) {
        stage_load(p0 - 2 * W + 1, sreg);
#pragma unroll
        for (int r = 0; r < W; ++r) rn[r] = (p0 - W - r >= 0) ? y[(size_t)(p0 - W - r) * 64] : 0.0;
      }
      const double* S = stg[b & 1];     // row p0 - r at staging row W - 1 - r
#pragma unroll
      for (int r = 0; r < W; ++r) {
        const int p = p0 - r;
        if (p >= 0) {
          const double* Ur = S + (W - 1 - r) * BW;
          // band entries of columns past Nx - 1 are zero, and so is the window before row Nx - 1
          double acc = rc[r], acc2 = 0.0;
#pragma unroll
          for (int k = 1; k <= W; ++k) {
            if (k & 1)
              acc -= Ur[W + k] * win[(r - k + W) % W];
            else
              acc2 -= Ur[W + k] * win[(r - k + W) % W];
          }
          acc = (acc + acc2) * Ur[W];
          win[r] = acc;
          w[(size_t)p * 64] = acc;
        }
      }
      if (more) {
        stage_store(stg[(b + 1) & 1], sreg);
#pragma unroll
        for (int r = 0; r < W; ++r) rc[r] = rn[r];
      }
      __syncthreads();
    }
  }
  if (on) {
    double* dst = out + (m * N + s) * Nx;
    for (int p = 0; p < Nx; ++p) dst[p] = w[(size_t)p * 64];
  }
}

// defect of the correction form: D[m][s] = (M + dT L)(F - U)[m][s]
__global__ __launch_bounds__(256) void ade_defect_kernel(const double* __restrict__ tab, int n,
                                                         const double* __restrict__ coef, double dT,
                                                         const int32_t* __restrict__ list, int N,
                                                         const double* __restrict__ Fv, const double* __restrict__ U,
                                                         double* __restrict__ D) {
  const int Nx = n * n;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  const int64_t li = blockIdx.z;
  if (p >= Nx) return;
  const int64_t m = list ? list[li] : li;
  const double a = coef[m];
  const int64_t row = (m * N + s) * Nx;
  const double* t = tab + (size_t)p * kTab;
  const int i = p % n, j = p / n;
  double acc = 0.0;
  for (int sl = 0; sl < 7; ++sl) {
    const int di = slot_di(sl), dj = slot_dj(sl);
    if (i + di < 0 || i + di >= n || j + dj < 0 || j + dj >= n) continue;
    const int q = p + di + n * dj;
    acc += (t[sl] + dT * (a * t[7 + sl] + t[14 + sl])) * (Fv[row + q] - U[row + q]);
  }
  D[row + p] = acc;
}

// (lambda_k M + dT L) q = p for (listed sample, bin k), in place in spec [M][K][Nx].
__global__ __launch_bounds__(64) void ade_shift_solve_kernel(const cplx* __restrict__ cfac, int Nx, int W, int K,
                                                             const int32_t* __restrict__ list,
                                                             cplx* __restrict__ spec) {
  extern __shared__ unsigned char smem[];
  cplx* v = reinterpret_cast<cplx*>(smem);     // [Nx]
  cplx* stage = v + Nx;                         // [kStage][2W+1]
  const int BW = 2 * W + 1;
  const int64_t li = blockIdx.x / K;
  const int k = blockIdx.x % K;
  const int64_t m = list ? list[li] : li;
  const int lane = threadIdx.x;
  const cplx* F = cfac + ((size_t)m * K + k) * Nx * BW;
  cplx* q = spec + ((size_t)m * K + k) * Nx;
  for (int p = lane; p < Nx; p += 64) v[p] = q[p];
  // forward: lane t < W holds y_{p-1-t}
  cplx win = cplx{0.0, 0.0};
  for (int c0 = 0; c0 < Nx; c0 += kStage) {
    const int nr = min(kStage, Nx - c0);
    __syncthreads();
    for (int e = lane; e < nr * BW; e += 64) stage[e] = F[(size_t)c0 * BW + e];
    __syncthreads();
    for (int r = 0; r < nr; ++r) {
      const int p = c0 + r;
      cplx term = cplx{0.0, 0.0};
      if (lane < W && p - 1 - lane >= 0) term = stage[r * BW + W - 1 - lane] * win;
#pragma unroll
      for (int off = 16; off >= 1; off >>= 1) {
        term.re += __shfl_xor(term.re, off, 64);
        term.im += __shfl_xor(term.im, off, 64);
      }
      const cplx yp = v[p] - term;
      const cplx up = cplx{__shfl_up(win.re, 1, 64), __shfl_up(win.im, 1, 64)};
      win = lane == 0 ? yp : up;
      if (lane == 0) v[p] = yp;
    }
  }
  // backward: lane t < W holds x_{p+1+t}
  win = cplx{0.0, 0.0};
  for (int c1 = Nx; c1 > 0; c1 -= kStage) {
    const int c0 = max(0, c1 - kStage);
    const int nr = c1 - c0;
    __syncthreads();
    for (int e = lane; e < nr * BW; e += 64) stage[e] = F[(size_t)c0 * BW + e];
    __syncthreads();
    for (int r = nr - 1; r >= 0; --r) {
      const int p = c0 + r;
      cplx term = cplx{0.0, 0.0};
      if (lane < W && p + 1 + lane < Nx) term = stage[r * BW + W + 1 + lane] * win;
#pragma unroll
      for (int off = 16; off >= 1; off >>= 1) {
        term.re += __shfl_xor(term.re, off, 64);
        term.im += __shfl_xor(term.im, off, 64);
      }
      const cplx xp = (v[p] - term) * stage[r * BW + W];
      const cplx up = cplx{__shfl_up(win.re, 1, 64), __shfl_up(win.im, 1, 64)};
      win = lane == 0 ? xp : up;
      if (lane == 0) v[p] = xp;
    }
  }
  __syncthreads();
  for (int p = lane; p < Nx; p += 64) q[p] = v[p];
}

int band_width_for(int n) { return ((n + 1) + 3) / 4 * 4; }

template <int W>
void launch_sweep_w(hipStream_t st, const double* tab, int n, const double* coef, const double* fac,
                    const int32_t* list, int64_t nlist, const AdeSweep& sw, int N, int J, double tau, double dT,
                    double* work) {
  const int lanes = kSweepLanes;
  const int waves = (sw.nsl + lanes - 1) / lanes;
  ade_sweep_kernel<W><<<(unsigned)(nlist * waves), 64, 0, st>>>(tab, n, coef, fac, list, sw.base, sw.u0,
                                                                sw.shift ? 1 : 0, sw.s_lo, sw.nsl, lanes, N, J,
                                                                tau, dT, work, sw.out);
}

}  // namespace

struct AdeState {
  klecgc_model mp;
  int64_t M = 0;
  int n = 0, Nx = 0, W = 0, K = 0;
  double dT = 0, dt = 0;
  const double* coef = nullptr;
  double* tab = nullptr;       // [Nx][kTab]
  double* fine = nullptr;      // [M][Nx][2W+1]
  double* coarse = nullptr;    // [M][Nx][2W+1] or null
  cplx* shifted = nullptr;     // [M][K][Nx][2W+1] or null
  int* bad = nullptr;          // [M][K + 2]
  double* work = nullptr;      // sweep work, [M][2][Nx][64]
  double* D = nullptr;         // defect [M][N][Nx]
  cplx* spec = nullptr;        // [M][K][Nx]
  SliceTables tb{};
};

void ade_initial_value(klecgc_ctx* ctx, const klecgc_model& mp, int64_t M, double* u0) {
  const int64_t tot = M * (int64_t)mp.n * mp.n;
  ade_u0_kernel<<<(unsigned)std::min<int64_t>((tot + 255) / 256, 65535), 256, 0, ctx->stream>>>(mp.n, M, u0);
  KC_LAUNCH_CHECK();
}

AdeState* ade_prepare(klecgc_ctx* ctx, const klecgc_model& mp, const double* c, int64_t M, bool need_coarse,
                      bool need_shifted) {
  auto* s = new AdeState;
  try {
    hipStream_t st = ctx->stream;
    s->mp = mp;
    s->M = M;
    s->n = mp.n;
    s->Nx = mp.n * mp.n;
    s->W = band_width_for(mp.n);
    s->K = model_bins(mp.N);
    s->dT = mp.T / mp.N;
    s->dt = s->dT / mp.J;
    s->coef = c;
    const int BW = 2 * s->W + 1;
    const size_t band = (size_t)s->Nx * BW;
    // small tables: node tables, slice tables, bad flags
    const size_t tab_b = sizeof(double) * (size_t)s->Nx * kTab;
    const size_t sl_b = sizeof(double) * 3 * (size_t)mp.N;
    const size_t bad_b = sizeof(int) * (size_t)M * (s->K + 2);
    char* sm = (char*)ctx->ws.get(WS_MODEL_SMALL, tab_b + sl_b + bad_b + 512);
    s->tab = (double*)sm;
    double* slt = (double*)(sm + tab_b);
    s->bad = (int*)(sm + tab_b + sl_b);
    KC_TRY_HIP(hipMemsetAsync(s->bad, 0, bad_b, st));
    s->tb = slice_tables(ctx, mp.N, mp.alpha, slt);
    ade_tables_kernel<<<(s->Nx + 127) / 128, 128, 0, st>>>(s->n, mp.beta, s->tab);
    KC_LAUNCH_CHECK();
    double* fb = (double*)ctx->ws.get(WS_MODEL_FAC, sizeof(double) * band * M * (need_coarse ? 2 : 1));
    s->fine = fb;
    s->coarse = need_coarse ? fb + band * M : nullptr;
    const size_t lds_real = sizeof(double) * ((size_t)(s->W + 1) * BW + s->W);
    ade_factor_kernel<double><<<(unsigned)M, 64, lds_real, st>>>(s->tab, s->n, s->W, c, 1, mp.N, 0.0, s->dt, 0,
                                                                 s->fine, s->bad);
    KC_LAUNCH_CHECK();
    if (need_coarse) {
      ade_factor_kernel<double><<<(unsigned)M, 64, lds_real, st>>>(s->tab, s->n, s->W, c, 1, mp.N, 0.0, s->dT, 0,
                                                                   s->coarse, s->bad + M);
      KC_LAUNCH_CHECK();
    }
    if (need_shifted) {
      s->shifted = (cplx*)ctx->ws.get(WS_MODEL_CFAC, sizeof(cplx) * band * M * s->K);
      const size_t lds_c = sizeof(cplx) * ((size_t)(s->W + 1) * BW + s->W);
      timed(ctx, KT_SHIFTED, [&] {
        ade_factor_kernel<cplx><<<(unsigned)(M * s->K), 64, lds_c, st>>>(
            s->tab, s->n, s->W, c, s->K, mp.N, std::pow(mp.alpha, 1.0 / mp.N), s->dT, 1, s->shifted, s->bad + 2 * M);
      });
      KC_LAUNCH_CHECK();
      s->D = (double*)ctx->ws.get(WS_MODEL_STATE, sizeof(double) * (size_t)M * mp.N * s->Nx);
      s->spec = (cplx*)ctx->ws.get(WS_MODEL_SPEC, sizeof(cplx) * (size_t)M * s->K * s->Nx);
    }
    const int waves = (mp.N + kSweepLanes - 1) / kSweepLanes;   // wavefronts per sample of the widest sweep
    s->work = (double*)ctx->ws.get(WS_MODEL_WORK,
                                   sizeof(double) * (size_t)M * waves * 2 * (s->Nx + 2 * (s->n + 1)) * 64);
  } catch (...) {
    delete s;
    throw;
  }
  return s;
}

void ade_release(AdeState* s) { delete s; }

int ade_bad_samples(klecgc_ctx* ctx, AdeState* s, std::vector<uint8_t>& bad) {
  const int64_t M = s->M;
  std::vector<int> h((size_t)M * (s->K + 2));
  KC_TRY_HIP(hipMemcpyAsync(h.data(), s->bad, sizeof(int) * h.size(), hipMemcpyDeviceToHost, ctx->stream));
  KC_TRY_HIP(hipStreamSynchronize(ctx->stream));
  bad.assign((size_t)M, 0);
  int any = 0;
  for (int64_t m = 0; m < M; ++m) {
    int b = h[m] | h[M + m];
    for (int k = 0; k < s->K; ++k) b |= h[2 * M + m * s->K + k];
    bad[m] = (uint8_t)(b != 0);
    any |= b;
  }
  return any;
}

void ade_sweep(klecgc_ctx* ctx, AdeState* s, const int32_t* list, int64_t nlist, const AdeSweep& sw) {
  if (nlist <= 0 || sw.nsl <= 0) return;
  KC_REQUIRE(sw.nsl <= 64, KC_EINVAL, "at most 64 slices per sweep");
  KC_REQUIRE(!sw.coarse || s->coarse, KC_EINVAL, "coarse factors not prepared");
  const double* fac = sw.coarse ? s->coarse : s->fine;
  const int J = sw.coarse ? 1 : s->mp.J;
  const double tau = sw.coarse ? s->dT : s->dt;
  hipStream_t st = ctx->stream;
  timed(ctx, KT_FINE, [&] {
    switch (s->W) {
#define KC_ADE_W(w) \
  case w:           \
    launch_sweep_w<w>(st, s->tab, s->n, s->coef, fac, list, nlist, sw, s->mp.N, J, tau, s->dT, s->work); break;
      KC_ADE_W(4)
      KC_ADE_W(8)
      KC_ADE_W(12)
      KC_ADE_W(16)
      KC_ADE_W(20)
      KC_ADE_W(24)
      KC_ADE_W(28)
      KC_ADE_W(32)
#undef KC_ADE_W
      default:
        throw Error{KC_EUNSUPPORTED, "grid too large for the banded model solver (n <= 31)"};
    }
  });
  KC_LAUNCH_CHECK();
}

void ade_correct(klecgc_ctx* ctx, AdeState* s, const int32_t* list, int64_t nlist, const double* Fv, double* U,
                 unsigned long long* maxima) {
  if (nlist <= 0) return;
  KC_REQUIRE(s->shifted, KC_EINVAL, "shifted factors not prepared");
  hipStream_t st = ctx->stream;
  const int N = s->mp.N;
  dim3 g((unsigned)((s->Nx + 255) / 256), (unsigned)N, (unsigned)nlist);
  timed(ctx, KT_DEFECT, [&] { ade_defect_kernel<<<g, 256, 0, st>>>(s->tab, s->n, s->coef, s->dT, list, N, Fv, U, s->D); });
  KC_LAUNCH_CHECK();
  timed(ctx, KT_FFT_FWD, [&] { launch_slice_dft(st, s->D, list, nlist, N, s->Nx, s->tb, s->spec); });
  const int BW = 2 * s->W + 1;
  const size_t lds = sizeof(cplx) * ((size_t)s->Nx + (size_t)kStage * BW);
  timed(ctx, KT_SHIFTED, [&] {
    ade_shift_solve_kernel<<<(unsigned)(nlist * s->K), 64, lds, st>>>(s->shifted, s->Nx, s->W, s->K, list, s->spec);
  });
  KC_LAUNCH_CHECK();
  timed(ctx, KT_FFT_INV, [&] { launch_slice_idft(st, s->spec, list, nlist, N, s->Nx, s->tb, U, true, maxima); });
}

static_assert(kMaxW == 32, "the shifted-solve window reduction spans 32 lanes");

}  // namespace kc
