// Fine propagator F (Algorithm 2 step 1): J backward-Euler steps per (sample, slice).
//
// One step of size tau solves (I + tau A) w_new = w + tau f (Section 3.1; Section 5 uses
// backward Euler for F and G).  Three implementations:
//  * 1D: direct tridiagonal (Thomas) solves in float64, one thread per system, the
//    factorisation tables built once per sample (the matrix is the same for every slice).
//  * 2D, float64: Jacobi-PCG, one work-group per system streaming its vectors.
//  * 2D, float32-refined: one work-group of up to 16 waves per system keeps the whole
//    system on the CU.  The float32 Krylov state (Jacobi-PCG on the full system, or CG on
//    the red-black reduced system) and the float32 scaled stencil coefficients live in
//    registers; neighbours cross lanes with DPP shifts and cross waves through LDS halo
//    rows.  Each step is solved for its increment and refined in float64: every pass forms
//    the true residual of the step equation in float64 with float64 coefficients from the
//    state and the increment, the float32 solve gives a correction and the increment takes
//    it in float64, until the residual meets inner_rtol * (|w|_inf + tau |f|) (plus the
//    float64 rounding floor).  With even n each residual sweep also applies the update
//    that precedes it (the close of the previous step, or the last pass's correction).
//  * 2D, multigrid-preconditioned: one work-group per system streams float32 vectors and
//    the V-cycle levels through device memory, for grids too large to stay on the CU.
#include <cmath>
#include <type_traits>

#include "common.h"
#include "fine_common.h"
#include "mg.h"
#include "reduce.h"
#include "xcd.h"

namespace kc {

namespace {

constexpr int kStreamThreads = 256;
// what the resident kernels' float64 residual sweep also does (column pairs): nothing, the
// update that closes the previous step, or the update by the last float32 pass
constexpr int kSweepPlain = 0, kSweepStart = 1, kSweepCorrect = 2;
#ifndef KC_RES128_NW
#define KC_RES128_NW 16
#endif


// ------------------------------------------------------------------------- 1D
__global__ void tri_factor_kernel(const double* __restrict__ a, int n, double c, int64_t M,
                                  double* __restrict__ tab) {
  int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const double* af = a + m * (n + 1);
  double* sub = tab + m * 3 * n;
  double* cp = sub + n;
  double* inv = cp + n;
  double prev = 0.0;
  for (int i = 0; i < n; ++i) {
    double aw = af[i], ae = af[i + 1];
    double diag = 1.0 + c * (aw + ae);
    double lo = (i > 0) ? -c * aw : 0.0;
    double up = (i < n - 1) ? -c * ae : 0.0;
    double iv = 1.0 / (diag - lo * prev);
    sub[i] = lo;
    inv[i] = iv;
    cp[i] = up * iv;
    prev = cp[i];
  }
}

__global__ void fine1d_kernel(const double* __restrict__ tab, int n, int J, double tauf,
                              StartRef sr, double* __restrict__ out, int64_t M, int N,
                              int skip_first, const uint8_t* __restrict__ active) {
  int64_t sys = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t m = sys / N;
  int s = (int)(sys % N);
  if (m >= M) return;
  if (active && !active[m]) return;
  if (skip_first && s == 0) return;
  const double* src = sr.row(m, s, N, n);
  double* w = out + sys * n;
  for (int i = 0; i < n; ++i) w[i] = src ? src[i] : 0.0;
  const double* sub = tab + m * 3 * n;
  const double* cp = sub + n;
  const double* inv = cp + n;
  for (int j = 0; j < J; ++j) {
    double prev = 0.0;
    for (int i = 0; i < n; ++i) {
      double d = (w[i] + tauf - sub[i] * prev) * inv[i];
      w[i] = d;
      prev = d;
    }
    for (int i = n - 2; i >= 0; --i) w[i] -= cp[i] * w[i + 1];
  }
}

// --------------------------------------------------------------- 2D helpers

// D^{-1/2} of M = I + c h^2 A (c = tau / h^2): d_p = 1 + c * (sum of the face coefficients of p)
// dinvf (nullable) receives the same values rounded to float32.
__global__ void dinv_kernel(const double* __restrict__ a, int n, double c, int64_t M,
                            double* __restrict__ dinv, float* __restrict__ dinvf) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t m = blockIdx.y;
  int64_t Nx = (int64_t)n * n;
  if (p >= Nx || m >= M) return;
  Grid2 g{n, (int64_t)n * (n + 1)};
  int i = (int)(p % n), j = (int)(p / n);
  const double* af = a + m * 2 * g.nx;
  double d = 1.0 + c * (af[g.fW(i, j)] + af[g.fE(i, j)] + af[g.fS(i, j)] + af[g.fN(i, j)]);
  const double v = 1.0 / sqrt(d);
  dinv[m * Nx + p] = v;
  if (dinvf) dinvf[m * Nx + p] = (float)v;
}

// float32 coefficients of the symmetrically Jacobi-scaled operator D^{-1/2} M D^{-1/2}:
// s_f = c a_f / sqrt(d_L d_R) on interior faces, 0 on boundary faces.
__global__ void scaled_faces_kernel(const double* __restrict__ a, const double* __restrict__ dinv,
                                    int n, double c, int64_t M, float* __restrict__ sf) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t m = blockIdx.y;
  int64_t nx = (int64_t)n * (n + 1);
  int64_t Fc = 2 * nx;
  if (f >= Fc || m >= M) return;
  int64_t Nx = (int64_t)n * n;
  const double* dv = dinv + m * Nx;
  float out = 0.f;
  if (f < nx) {
    int j = (int)(f / (n + 1)), fi = (int)(f % (n + 1));
    if (fi >= 1 && fi <= n - 1)
      out = (float)(c * a[m * Fc + f] * dv[(int64_t)j * n + fi - 1] * dv[(int64_t)j * n + fi]);
  } else {
    int64_t g = f - nx;
    int fj = (int)(g / n), i = (int)(g % n);
    if (fj >= 1 && fj <= n - 1)
      out = (float)(c * a[m * Fc + f] * dv[(int64_t)(fj - 1) * n + i] * dv[(int64_t)fj * n + i]);
  }
  sf[m * Fc + f] = out;
}



// --------------------------------------------------- 2D streaming float64 PCG
// One work-group per (sample, slice) system; x is the state row of `out`, r/p/q live
// in per-system scratch.  Jacobi preconditioner z = d^{-1} r (d^{-1} = dinv^2).
__global__ __launch_bounds__(kStreamThreads) void fine2d_pcg64_kernel(
    const double* __restrict__ a, const double* __restrict__ dinv, int n, double c, double tauf,
    int J, double tol, int maxit, StartRef sr, double* __restrict__ out, double* __restrict__ scr,
    int64_t M, int N, int skip_first, const uint8_t* __restrict__ active, int* __restrict__ flag,
    unsigned long long* __restrict__ cnt) {
  __shared__ double slots[3 * (kStreamThreads / 64)];
  unsigned long long tot_it = 0, max_it = 0, missed = 0;
  // the slices of a sample share its coefficients (and scaled forms): XCD-major order
  // keeps them under one L2
  const int64_t sys = xcd_major(blockIdx.x, gridDim.x);
  const int64_t m = sys / N;
  const int s = (int)(sys % N);
  if (active && !active[m]) return;
  if (skip_first && s == 0) return;
  const int64_t Nx = (int64_t)n * n;
  Grid2 g{n, (int64_t)n * (n + 1)};
  const double* af = a + m * 2 * g.nx;
  const double* dv = dinv + m * Nx;
  double* x = out + sys * Nx;
  double* R = scr + sys * 3 * Nx;
  double* P = R + Nx;
  double* Q = P + Nx;
  const double* src = sr.row(m, s, N, Nx);
  double dmx[1] = {0.0};
  const bool mxd[1] = {true};
  for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
    x[p] = src ? src[p] : 0.0;
    dmx[0] = nanmax(dmx[0], 1.0 / (dv[p] * dv[p]));
  }
  block_reduce<1>(dmx, mxd, slots);
  const double dmax = dmx[0];
  for (int step = 0; step < J; ++step) {
    // r = (x + tau f) - M x, initial guess x (the previous state)
    double acc[3] = {0.0, 0.0, 0.0};
    const bool mx3[3] = {false, true, true};
    for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
      int i = (int)(p % n), j = (int)(p / n);
      double r = tauf - c * stencil64(af, x, g, i, j);
      double z = r * dv[p] * dv[p];
      R[p] = r;
      P[p] = z;
      acc[0] += r * z;
      acc[1] = nanmax(acc[1], fabs(r));
      acc[2] = nanmax(acc[2], fabs(x[p]));
    }
    block_reduce<3>(acc, mx3, slots);
    double rz = acc[0], rmax = acc[1];
    const double target = residual_target(tol, acc[2], tauf, dmax);
    int it = 0;
    while (rmax > target && it < maxit) {
      double pq[1] = {0.0};
      const bool mx1[1] = {false};
      for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
        int i = (int)(p % n), j = (int)(p / n);
        double q = P[p] + c * stencil64(af, P, g, i, j);
        Q[p] = q;
        pq[0] += P[p] * q;
      }
      block_reduce<1>(pq, mx1, slots);
      const double alpha = rz / pq[0];
      double acc2[2] = {0.0, 0.0};
      const bool mx2[2] = {false, true};
      for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
        x[p] += alpha * P[p];
        double r = R[p] - alpha * Q[p];
        R[p] = r;
        acc2[0] += r * r * dv[p] * dv[p];
        acc2[1] = nanmax(acc2[1], fabs(r));
      }
      block_reduce<2>(acc2, mx2, slots);
      const double beta = acc2[0] / rz;
      rz = acc2[0];
      rmax = acc2[1];
      for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) P[p] = R[p] * dv[p] * dv[p] + beta * P[p];
      __syncthreads();
      ++it;
    }
    if (rmax > target) {
      ++missed;
      if (threadIdx.x == 0) atomicOr(flag, 1);
    }
    tot_it += it;
    max_it = it > (int)max_it ? it : max_it;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&cnt[0], tot_it);
    atomicAdd(&cnt[1], (unsigned long long)J);
    atomicAdd(&cnt[2], (unsigned long long)J);
    atomicMax(&cnt[3], max_it);
    atomicAdd(&cnt[5], missed);
  }
}

// ---------------------------------------------- 2D resident float32-refined PCG
// Tile ownership: wave w of NW owns grid rows [w*RPW, (w+1)*RPW); lane l owns columns
// [l*CPL, (l+1)*CPL).  Padded unknowns (outside the n x n grid) carry zero
// coefficients and stay zero.

// DPP helpers (gfx9 wavefront shifts; bound_ctrl fills the shifted-in lane with 0)
template <int CTRL>
__device__ __forceinline__ float dppf(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_west(float v) { return dppf<0x138>(v); }   // wave_shr:1
__device__ __forceinline__ float from_east(float v) { return dppf<0x130>(v); }   // wave_shl:1

// float64 lane shift (both halves moved by DPP; the shifted-in lane reads 0.0)
template <int CTRL>
__device__ __forceinline__ double dppd(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double2 ld2(const double* p) { return *reinterpret_cast<const double2*>(p); }

// float64 DPP move restricted to the rows in ROWMASK (other rows, and lanes without a source,
// read 0.0)
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dppd_rows(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWMASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xf, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Maximum within each 16-lane row, left in the row's lane 15 (row shifts by 1, 2, 4, 8 with
// 0.0 shifted in: the values are non-negative, and a NaN anywhere stays NaN).
__device__ __forceinline__ double row_max_dpp(double x) {
  x = nanmax(x, dppd_rows<0x111, 0xf>(x));
  x = nanmax(x, dppd_rows<0x112, 0xf>(x));
  x = nanmax(x, dppd_rows<0x114, 0xf>(x));
  x = nanmax(x, dppd_rows<0x118, 0xf>(x));
  return x;
}

// Maxima over the work-group of K non-negative float64 values per thread (NaN if any is NaN),
// returned uniform in every lane.  Within a wave by DPP (rows, then two row broadcasts into
// lane 63), one slot per wave, a barrier, then lanes 0..NW-1 reduce the slots within row 0
// and lane 15's result is read back as a scalar.  slots: K * NW doubles; the closing barrier
// lets the next call reuse them.
template <int NW, int K>
__device__ __forceinline__ void block_max_nn(double (&v)[K], double* slots, int lane, int wave) {
  static_assert(NW <= 16, "one slot per lane of row 0");
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x = row_max_dpp(v[k]);
    x = nanmax(x, dppd_rows<0x142, 0xa>(x));   // row_bcast:15 into rows 1 and 3
    x = nanmax(x, dppd_rows<0x143, 0xc>(x));   // row_bcast:31 into rows 2 and 3
    if (lane == 63) slots[k * NW + wave] = x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double x = row_max_dpp(lane < NW ? slots[k * NW + lane] : 0.0);
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_readlane((int)b, 15);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 15);
    v[k] = __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
  }
  __syncthreads();
}

__device__ __forceinline__ void st2(double* p, double x, double y) {
  *reinterpret_cast<double2*>(p) = make_double2(x, y);
}

// Butterfly sum within each 16-lane row by DPP: every lane of a row ends with the row's
// sum (the same bits in all 16 lanes, since each step adds two equal partial sums).
__device__ __forceinline__ float row_sum_dpp(float v) {
  v += dppf<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dppf<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dppf<0x141>(v);   // row_half_mirror
  v += dppf<0x140>(v);   // row_mirror
  return v;
}

// DPP move restricted to the rows in ROWMASK; other lanes read 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dppf_rows(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWMASK, 0xf, false));
}

// Sum over the work-group of NW <= 16 waves, uniform result.  Each wave reduces its four
// 16-lane rows and writes the four row sums; after the barrier lane l of every wave
// reads row sum l, the rows reduce again, and two row broadcasts (row 0 into row 1,
// rows 0..1 into rows 2..3) collect the total in lane 63.  slots: 4 NW floats.  One
// barrier: consecutive sums must alternate between two slot arrays unless another
// barrier separates them.
template <int NW>
__device__ __forceinline__ float block_sum_f(float v, float* slots, int lane, int wave) {
  static_assert(NW <= 16, "one row sum per lane");
  v = row_sum_dpp(v);
  if ((lane & 15) == 0) slots[wave * 4 + (lane >> 4)] = v;
  __syncthreads();
  float acc = lane < 4 * NW ? slots[lane] : 0.f;
  acc = row_sum_dpp(acc);
  acc += dppf_rows<0x142, 0xa>(acc);   // row_bcast:15 into rows 1 and 3
  acc += dppf_rows<0x143, 0xc>(acc);   // row_bcast:31 into rows 2 and 3
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, acc), 63));
}

template <int NW, int CPL, int RPW>
struct Resident {
  static constexpr int ROWW = 64 * CPL;   // halo row width per wave

  // Q = P - sum_f s_f P_nbr (scaled operator with unit diagonal); returns the lane's P.Q.
  // EW[s][t] is the negated coefficient -s_f of the face west of column t, NS[s][t] that
  // of the face south of row s (stored negated so each neighbour term is one
  // multiply-add whose lane-shifted operand can ride on the instruction as DPP).  The faces east of the lane's last column and north of the wave's
  // last row belong to the neighbouring lane / wave, which supplies the products
  // coefficient * value: across lanes by a DPP shift, across waves through LDS halos.
  // The halos hold the previous iteration's r and p rows; the current p row is
  // r + beta p, formed here (the halo exchange rides on the reduction barrier).
  static __device__ __forceinline__ float matvec(const float (&P)[RPW][CPL], float (&Q)[RPW][CPL],
                                                 const float (&EW)[RPW][CPL],
                                                 const float (&NS)[RPW][CPL],
                                                 const float* hr_top, const float* hp_top,
                                                 const float* hr_bot, const float* hp_bot,
                                                 float beta, int lane, int wave) {
    float pq = 0.f;
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      const float wv = from_west(P[s][CPL - 1]);
      const float ep = from_east(EW[s][0] * P[s][0]);
#pragma unroll
      for (int t = 0; t < CPL; ++t) {
        // terms within the lane first; the lane-shifted ones last, where they feed an
        // accumulating multiply-add / add that can take them as a DPP operand
        float q = P[s][t];
        if (t > 0) q = fmaf(EW[s][t], P[s][t - 1], q);
        if (t < CPL - 1) q = fmaf(EW[s][t + 1], P[s][t + 1], q);
        float down;
        if (s == 0) {
          const int h = (wave - 1) * ROWW + lane * CPL + t;
          down = (wave > 0) ? fmaf(beta, hp_bot[h], hr_bot[h]) : 0.f;
        } else {
          down = P[s - 1][t];
        }
        q = fmaf(NS[s][t], down, q);
        if (s == RPW - 1) {
          const int h = (wave + 1) * ROWW + lane * CPL + t;
          q += (wave < NW - 1) ? fmaf(beta, hp_top[h], hr_top[h]) : 0.f;
        } else {
          q = fmaf(NS[s + 1][t], P[s + 1][t], q);
        }
        if (t == 0) q = fmaf(EW[s][0], wv, q);
        if (t == CPL - 1) q += ep;
        Q[s][t] = q;
        pq = fmaf(P[s][t], q, pq);
      }
    }
    return pq;
  }

  // top: negated south-face coefficient times the row-0 value (the wave below the
  // boundary needs it as its northern term); bot: the last row's values.
  static __device__ __forceinline__ void store_halo(const float (&Rv)[RPW][CPL], const float (&Pv)[RPW][CPL],
                                                    const float (&NS)[RPW][CPL], float* hr_top,
                                                    float* hp_top, float* hr_bot, float* hp_bot,
                                                    int lane, int wave) {
#pragma unroll
    for (int t = 0; t < CPL; ++t) {
      const int h = wave * ROWW + lane * CPL + t;
      hr_top[h] = NS[0][t] * Rv[0][t];
      hp_top[h] = NS[0][t] * Pv[0][t];
      hr_bot[h] = Rv[RPW - 1][t];
      hp_bot[h] = Pv[RPW - 1][t];
    }
  }
};

// Red-black reduced system for two columns per lane (Section 3.1 step equation, Jacobi-
// scaled: I + N with N the negated scaled couplings, which join only nodes of opposite
// colour (i + j) mod 2).  With even nodes e and odd nodes o, eliminating o leaves
// S x_e = b_e - N_eo b_o with S = I - N_eo N_oe, whose condition number is about a quarter
// of that of I + N (eigenvalues 1 - mu^2 against 1 +- mu), so CG needs about half the
// iterations on half the unknowns; then x_o = b_o - N_oe x_e.  Wave w owns rows
// [w RPW, (w+1) RPW) with RPW even, so row s of a lane has its even node in column
// i0 + (s & 1) and its odd node in the other one, and the direction of each lane shift is
// fixed per row.  Halo arrays hold one value per lane and wave: "bot" the wave's last row
// (read by the wave above), "top" the wave's first row times its south-face coupling (read
// by the wave below).
template <int NW, int RPW>
struct RedBlack {
  static_assert(RPW % 2 == 0, "rows of both parities in every wave");
  static constexpr int HW = 64 * NW;

  // T = N_oe P (odd node of every row).  The neighbouring waves' boundary rows of P arrive
  // as r + beta p from the halos of the previous iteration (as in the full-system kernel).
  static __device__ __forceinline__ void gather_odd(const float (&P)[RPW], float (&T)[RPW],
                                                    const float (&EW)[RPW][2], const float (&NS)[RPW][2],
                                                    const float* hr_top, const float* hp_top,
                                                    const float* hr_bot, const float* hp_bot, float beta,
                                                    int lane, int wave) {
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      float t;
      if ((s & 1) == 0) {   // odd node in column i0 + 1
        const float south = s > 0 ? P[s - 1]
                                  : (wave > 0 ? fmaf(beta, hp_bot[(wave - 1) * 64 + lane], hr_bot[(wave - 1) * 64 + lane])
                                              : 0.f);
        t = EW[s][1] * P[s];
        t = fmaf(NS[s][1], south, t);
        t = fmaf(NS[s + 1][1], P[s + 1], t);
        t += from_east(EW[s][0] * P[s]);
      } else {              // odd node in column i0
        t = EW[s][1] * P[s];
        t = fmaf(NS[s][0], P[s - 1], t);
        if (s < RPW - 1)
          t = fmaf(NS[s + 1][0], P[s + 1], t);
        else
          t += wave < NW - 1 ? fmaf(beta, hp_top[(wave + 1) * 64 + lane], hr_top[(wave + 1) * 64 + lane]) : 0.f;
        t = fmaf(EW[s][0], from_west(P[s]), t);
      }
      T[s] = t;
    }
  }

  // Q = P - N_eo T (even node of every row); returns the lane's P.Q.
  static __device__ __forceinline__ float gather_even(const float (&P)[RPW], const float (&T)[RPW],
                                                      float (&Q)[RPW], const float (&EW)[RPW][2],
                                                      const float (&NS)[RPW][2], const float* ht_top,
                                                      const float* ht_bot, int lane, int wave) {
    float pq = 0.f;
#pragma unroll
    for (int s = 0; s < RPW; ++s) {
      float u;
      if ((s & 1) == 0) {   // even node in column i0
        const float south = s > 0 ? T[s - 1] : (wave > 0 ? ht_bot[(wave - 1) * 64 + lane] : 0.f);
        u = EW[s][1] * T[s];
        u = fmaf(NS[s][0], south, u);
        u = fmaf(NS[s + 1][0], T[s + 1], u);
        u = fmaf(EW[s][0], from_west(T[s]), u);
      } else {              // even node in column i0 + 1
        u = EW[s][1] * T[s];
        u = fmaf(NS[s][1], T[s - 1], u);
        if (s < RPW - 1)
          u = fmaf(NS[s + 1][1], T[s + 1], u);
        else
          u += wave < NW - 1 ? ht_top[(wave + 1) * 64 + lane] : 0.f;
        u += from_east(EW[s][0] * T[s]);
      }
      const float q = P[s] - u;
      Q[s] = q;
      pq = fmaf(P[s], q, pq);
    }
    return pq;
  }

  // halo rows of an even-node vector pair (R, P): last rows and first rows times the
  // coupling to the odd node below them (column i0: row 0 is even)
  static __device__ __forceinline__ void store_even_halo(const float (&Rv)[RPW], const float (&Pv)[RPW],
                                                         const float (&NS)[RPW][2], float* hr_top, float* hp_top,
                                                         float* hr_bot, float* hp_bot, int lane, int wave) {
    const int h = wave * 64 + lane;
    hr_bot[h] = Rv[RPW - 1];
    hp_bot[h] = Pv[RPW - 1];
    hr_top[h] = NS[0][0] * Rv[0];
    hp_top[h] = NS[0][0] * Pv[0];
  }

  // halo rows of an odd-node vector (row 0's odd node is in column i0 + 1)
  static __device__ __forceinline__ void store_odd_halo(const float (&Tv)[RPW], const float (&NS)[RPW][2],
                                                        float* ht_top, float* ht_bot, int lane, int wave) {
    const int h = wave * 64 + lane;
    ht_bot[h] = Tv[RPW - 1];
    ht_top[h] = NS[0][1] * Tv[0];
  }
};

typedef float __attribute__((address_space(3))) lds_float;   // a pointer into LDS

struct RbPassOut {
  int it;            // reduced-system CG iterations
  int capped;        // the iteration cap ended the pass above its stop
  long long cycles;  // shader clocks inside the Krylov loop
};

// One float32 correction pass of the red-black reduced solve (see RedBlack).  In: the pass's
// right-hand side D^{-1/2} r / sig in xs (scaled by fis here).  Out: the correction of every
// owned node in xs.  Called by every thread of the work-group.  Inlined: as a call it would
// save and restore the ~40 callee-saved VGPRs it uses (v40-47, v56-63, ...) on every pass,
// some 10 KB of scratch traffic per wave; inlined, its lane and row indices are re-formed at
// each pass (opaque below), so no address arithmetic is hoisted out of the caller's loops
// into scratch across the Krylov loop.
template <int NW, int RPW>
__device__ __forceinline__ RbPassOut rb_pass(lds_float* xs_l, float fis, const float* __restrict__ sfm,
                                                     int n, int64_t gnx, float rel, int maxit, lds_float* hr_top_l,
                                                     lds_float* hp_top_l, lds_float* hr_bot_l, lds_float* hp_bot_l,
                                                     lds_float* ht_top_l, lds_float* ht_bot_l, lds_float* fs0_l,
                                                     lds_float* fs1_l) {
  using RBS = RedBlack<NW, RPW>;
  float* xs = (float*)xs_l;
  float *hr_top = (float*)hr_top_l, *hp_top = (float*)hp_top_l, *hr_bot = (float*)hr_bot_l, *hp_bot = (float*)hp_bot_l;
  float *ht_top = (float*)ht_top_l, *ht_bot = (float*)ht_bot_l, *fs0 = (float*)fs0_l, *fs1 = (float*)fs1_l;
  int lane = threadIdx.x & 63;
  int wave = threadIdx.x >> 6;
  asm volatile("" : "+v"(lane), "+v"(wave));
  wave = __builtin_amdgcn_readfirstlane(wave);   // uniform: halo branches on the scalar unit
  const int j0 = wave * RPW, i0 = lane * 2;
  // negated scaled couplings (0 on boundary faces and outside the grid)
  float EW[RPW][2], NS[RPW][2];
  if ((n & 1) == 0) {
    // even n: one 8-byte load per row and kind, every byte of the touched lines used.  The
    // y-face pair (i0, i0 + 1) is aligned in every row; the x-face pair (i0, i0 + 1) only on
    // even rows (rows hold n + 1 faces), so odd rows load (i0 + 1, i0 + 2) and take face i0
    // from the western lane.  Clamped indices keep lanes and rows outside the grid in bounds.
    const bool lane_ok = i0 < n;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int j = j0 + r;
      const bool ok = j < n && lane_ok;
      // rows outside the grid read a row of the same parity (the pair stays 8-byte aligned)
      const int jc = j < n ? j : ((r & 1) ? n - 1 : n - 2), ic = lane_ok ? i0 : 0;
      const float2 X2 = *reinterpret_cast<const float2*>(sfm + (int64_t)jc * (n + 1) + ic + (r & 1));
      const float2 Y2 = *reinterpret_cast<const float2*>(sfm + gnx + (int64_t)jc * n + ic);
      const float e0 = (r & 1) ? from_west(X2.y) : X2.x;   // face west of column i0
      const float e1 = (r & 1) ? X2.x : X2.y;              // face between i0 and i0 + 1
      EW[r][0] = (ok && i0 >= 1) ? -e0 : 0.f;
      EW[r][1] = (ok && i0 + 1 <= n - 1) ? -e1 : 0.f;
      NS[r][0] = (ok && j >= 1) ? -Y2.x : 0.f;
      NS[r][1] = (ok && j >= 1) ? -Y2.y : 0.f;
    }
  } else {
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int j = j0 + r;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int col = i0 + t;
        EW[r][t] = (j < n && col >= 1 && col <= n - 1) ? -sfm[(int64_t)j * (n + 1) + col] : 0.f;
        NS[r][t] = (col < n && j >= 1 && j <= n - 1) ? -sfm[gnx + (int64_t)j * n + col] : 0.f;
      }
    }
  }
  // right-hand side b split by colour, then the reduced right-hand side R = b_e - N_eo b_o
  // (the odd values of the boundary rows through the halos)
  float Be[RPW], Bo[RPW], Xr[RPW], Rr[RPW], Pr[RPW], Qr[RPW], Tr[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    const int j = j0 + r;
    const int ce = i0 + (r & 1), co = i0 + 1 - (r & 1);
    Be[r] = (j < n && ce < n) ? xs[j * n + ce] * fis : 0.f;
    Bo[r] = (j < n && co < n) ? xs[j * n + co] * fis : 0.f;
  }
  RBS::store_odd_halo(Bo, NS, ht_top, ht_bot, lane, wave);
  __syncthreads();
  (void)RBS::gather_even(Be, Bo, Rr, EW, NS, ht_top, ht_bot, lane, wave);
  float rr = 0.f;
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    Pr[r] = Rr[r];
    Xr[r] = 0.f;
    rr = fmaf(Rr[r], Rr[r], rr);
  }
  RBS::store_even_halo(Rr, Pr, NS, hr_top, hp_top, hr_bot, hp_bot, lane, wave);
  rr = block_sum_f<NW>(rr, fs1, lane, wave);
  // the odd residual of the full system is zero after the back-substitution, so the reduced
  // residual is the full one
  const float stop = rel * rel * rr;
  float beta = 0.f;
  int it = 0;
  const long long t0 = clock64();
  while (rr > stop && it < maxit) {
    RBS::gather_odd(Pr, Tr, EW, NS, hr_top, hp_top, hr_bot, hp_bot, beta, lane, wave);
    RBS::store_odd_halo(Tr, NS, ht_top, ht_bot, lane, wave);
    __syncthreads();
    float pq = RBS::gather_even(Pr, Tr, Qr, EW, NS, ht_top, ht_bot, lane, wave);
    pq = block_sum_f<NW>(pq, fs0, lane, wave);
    // CG scalars through the hardware reciprocal (about 1 ulp)
    const float alpha = rr * __builtin_amdgcn_rcpf(pq);
    float rn = 0.f;
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      Xr[r] = fmaf(alpha, Pr[r], Xr[r]);
      Rr[r] = fmaf(-alpha, Qr[r], Rr[r]);
      rn = fmaf(Rr[r], Rr[r], rn);
    }
    RBS::store_even_halo(Rr, Pr, NS, hr_top, hp_top, hr_bot, hp_bot, lane, wave);
    rn = block_sum_f<NW>(rn, fs1, lane, wave);
    beta = rn * __builtin_amdgcn_rcpf(rr);
    rr = rn;
#pragma unroll
    for (int r = 0; r < RPW; ++r) Pr[r] = fmaf(beta, Pr[r], Rr[r]);
    ++it;
  }
  const long long cycles = clock64() - t0;
  // back-substitution x_o = b_o - N_oe x_e (even halo rows of x, beta = 0), then the whole
  // correction into the owners' xs entries
  RBS::store_even_halo(Xr, Xr, NS, hr_top, hp_top, hr_bot, hp_bot, lane, wave);
  __syncthreads();
  RBS::gather_odd(Xr, Tr, EW, NS, hr_top, hp_top, hr_bot, hp_bot, 0.f, lane, wave);
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    const int j = j0 + r;
    const int ce = i0 + (r & 1), co = i0 + 1 - (r & 1);
    if (j < n && ce < n) xs[j * n + ce] = Xr[r];
    if (j < n && co < n) xs[j * n + co] = Bo[r] - Tr[r];
  }
  return RbPassOut{it, (it >= maxit && rr > stop) ? 1 : 0, cycles};
}

// LDS: xs[n*n + 2] float32 staging tile of the whole system (+ a spare word pair for lanes
// outside the grid), halo rows, reduction slots.
// RB: the float32 solve runs CG on the red-black reduced system (CPL == 2), else Jacobi-PCG
// on the full system.
// A work-group's solver counters over the systems it has solved.
struct ResTally {
  unsigned long long its = 0, passes = 0, max_it = 0, missed = 0, steps = 0;
  long long cg_cycles = 0;
  bool fail = false;
};

// Thread 0 adds a work-group's counters to the status block (flag, cnt).
__device__ __forceinline__ void report_tally(const ResTally& tl, long long t_start, int* flag,
                                             unsigned long long* cnt) {
  if (threadIdx.x != 0) return;
  if (tl.fail) atomicOr(flag, 1);
  atomicAdd(&cnt[0], tl.its);
  atomicAdd(&cnt[1], tl.passes);
  atomicAdd(&cnt[2], tl.steps);
  atomicMax(&cnt[3], tl.max_it);
  atomicAdd(&cnt[5], tl.missed);
  atomicAdd(&cnt[8], (unsigned long long)(clock64() - t_start));
  atomicAdd(&cnt[9], (unsigned long long)tl.cg_cycles);
}

// J implicit steps of one (sample m, slice) system by the whole work-group: the sample's
// faces a, scaled faces sf, D^{-1/2} (float64 dinv, float32 dinvf) at their [M] bases, the
// start row src (nullptr: zero), the result row w, and two Nx rows of scratch (inc, incp)
// for the current and the previous step's increment.
template <int NW, int CPL, int RPW, bool RB>
__device__ __forceinline__ void resident_system(
    const double* __restrict__ a, const float* __restrict__ sf, const double* __restrict__ dinv,
    const float* __restrict__ dinvf, int n, double c, double tauf, int J, double tol, float pcg_rtol,
    int maxit, const double* __restrict__ src, double* __restrict__ w, double* __restrict__ inc,
    double* __restrict__ incp, int64_t m, ResTally& tally) {
  using RS = Resident<NW, CPL, RPW>;
  long long t_cg = 0;
  extern __shared__ float xs[];                       // [n*n + 2]
  __shared__ float hr_top[NW * RS::ROWW], hp_top[NW * RS::ROWW];
  __shared__ float hr_bot[NW * RS::ROWW], hp_bot[NW * RS::ROWW];
  __shared__ float ht_top[RB ? NW * 64 : 1], ht_bot[RB ? NW * 64 : 1];   // odd-node halos (RB)
  static_assert(!RB || CPL == 2, "the red-black solve pairs two columns per lane");
  __shared__ float fslots[2][4 * NW];
  __shared__ double dslots[4 * NW];
  unsigned long long tot_it = 0, tot_pass = 0, max_it = 0, missed = 0;
  const int lane = threadIdx.x & 63;
  // uniform across the wave: its rows' indices, tests and offsets go to the scalar unit
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int64_t Nx = (int64_t)n * n;
  Grid2 g{n, (int64_t)n * (n + 1)};
  const int64_t Fc = 2 * g.nx;
  const double* af = a + m * Fc;
  const float* sfm = sf + m * Fc;
  const double* dv = dinv + m * Nx;
  const float* dvf = dinvf + m * Nx;   // the same, float32: scaling of float32 quantities
  const int j0 = wave * RPW;
  const int i0 = lane * CPL;

  // negated scaled coefficients into registers (0 on boundary faces and outside the grid)
  float EW[RPW][CPL];
  float NS[RPW][CPL];
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    int j = j0 + r;
#pragma unroll
    for (int t = 0; t < CPL; ++t) {
      int col = i0 + t;
      EW[r][t] = (j < n && col >= 1 && col <= n - 1) ? -sfm[(int64_t)j * (n + 1) + col] : 0.f;
      NS[r][t] = (col < n && j >= 1 && j <= n - 1) ? -sfm[g.nx + (int64_t)j * n + col] : 0.f;
    }
  }

  double dmx[1] = {0.0};
  for (int64_t p = threadIdx.x; p < Nx; p += blockDim.x) {
    w[p] = src ? src[p] : 0.0;
    inc[p] = 0.0;
    incp[p] = 0.0;
    dmx[0] = nanmax(dmx[0], 1.0 / (dv[p] * dv[p]));
  }
  block_max_nn<NW, 1>(dmx, dslots, lane, wave);   // also orders the copy before the first stencil
  const double dmax = dmx[0];

  float X[RPW][CPL], R[RPW][CPL], P[RPW][CPL], Q[RPW][CPL];
  bool fail = false;
  // owned nodes per group of the float64 loops (residual sweep; increment / state updates)
  constexpr int KG = RPW * CPL < 4 ? RPW * CPL : 4;
  constexpr int KU = RPW * CPL < 8 ? RPW * CPL : 8;
  // column pairs per lane, 16-byte aligned in every row (even n)
  const bool pairs = CPL == 2 && (n & 1) == 0;
  constexpr int KR = 4;   // rows per group of the paired update loops
  static_assert((RPW * CPL) % KG == 0 && (RPW * CPL) % KU == 0, "whole groups");

  // float64 residual of the step equation (I + tau A) w_{j+1} = w_j + tau f at
  // w_j + inc:  tau f - tau A (w_j + inc) - inc, for the nodes this thread owns; it also
  // writes the unnormalised float32 right-hand side D^{-1/2} r of the next pass to xs.
  // acc: max |r|, max |w_j + inc|, max D^{-1/2} |r| over the work-group.
  // With column pairs the sweep can also finish the update that precedes it, on each row
  // as it is read (the state is then read once instead of twice):
  //  * MODE kSweepStart, the sweep that opens step j >= 1: memory holds w_{j-1}, its
  //    final increment and the one before; a row becomes w_j = w_{j-1} + inc and the
  //    starting increment ka inc + kb inc_prev, written back with inc as the new previous
  //    increment;
  //  * MODE kSweepCorrect, the sweep after a float32 pass: inc += ka D^{-1/2} x, with the
  //    pass's solution x in xs.
  auto residual = [&](double (&acc)[3], auto mode, double ka, double kb) {
    constexpr int MODE = decltype(mode)::value;
    constexpr bool FUSED = MODE != kSweepPlain;
    acc[0] = acc[1] = acc[2] = 0.0;
    if (pairs) {
      // A lane's two columns (i0, i0 + 1) together: 16-byte loads of w, inc, D^{-1/2} and
      // the y-faces use every byte of the cache lines a wave touches (two 8-byte loads
      // with a 16-byte lane stride would each touch twice the lines for half the data);
      // the west / east neighbour columns come from the adjacent lanes by DPP.
      const bool hw0 = i0 > 0, he1 = i0 + 1 < n - 1;
      const bool lane_ok = i0 < n;
      const int ic = lane_ok ? i0 : 0;   // clamped: every load in bounds
      const double2 zero2 = make_double2(0.0, 0.0);
      double bad = 0.0;
      // rows are walked upwards with a window of three rows of w and inc (south, current,
      // north) and the south y-faces carried over, so each row loads only its north row
      // FUSED: the update of the pair at q (in the grid); Iold: the increment it held
      auto advance = [&](int64_t q, double2& Wv, double2& Iv, double2& Iold) {
        const double2 w0 = ld2(w + q), i1 = ld2(inc + q);
        if constexpr (MODE == kSweepStart) {
          const double2 i2 = ld2(incp + q);
          Wv = make_double2(w0.x + i1.x, w0.y + i1.y);
          Iv = make_double2(ka * i1.x + kb * i2.x, ka * i1.y + kb * i2.y);
        } else {
          const float2 Df = *reinterpret_cast<const float2*>(dvf + q);
          const float2 Xv = *reinterpret_cast<const float2*>(xs + q);
          Wv = w0;
          Iv = make_double2(i1.x + ka * (double)Df.x * (double)Xv.x, i1.y + ka * (double)Df.y * (double)Xv.y);
        }
        Iold = i1;
      };
      // FUSED: the updated pair at q written back
      auto write_back = [&](int64_t q, const double2& Wv, const double2& Iv, const double2& Iold) {
        if constexpr (MODE == kSweepStart) {
          st2(w + q, Wv.x, Wv.y);
          st2(incp + q, Iold.x, Iold.y);
        }
        st2(inc + q, Iv.x, Iv.y);
      };
      double2 Ws, Is, Wc, Ic, FSc;
      double2 Wh, Ih;   // FUSED: the first row of the next wave (north halo of the last row)
      {
        const bool ok0 = j0 < n && lane_ok;
        const int jc = ok0 ? j0 : 0;
        const int64_t p = (int64_t)jc * n + ic;
        const bool hs = ok0 && jc > 0;
        const int64_t ps = hs ? p - n : p;
        double2 ws, is;
        if constexpr (FUSED) {
          // offsets re-formed at every sweep (opaque to loop-invariant hoisting, whose
          // nine 64-bit addresses would live in scratch)
          int64_t q0 = p, qs = ps, qh = j0 + RPW < n && lane_ok ? (int64_t)(j0 + RPW) * n + ic : p;
          asm volatile("" : "+v"(q0), "+v"(qs), "+v"(qh));
          double2 I0, Ix;
          advance(q0, Wc, Ic, I0);
          advance(qs, ws, is, Ix);
          advance(qh, Wh, Ih, Ix);
          // the rows a wave shares with its neighbours (its first and last, their south
          // and north halos; in xs too) are all read, and the loads complete, before any
          // is written
          __builtin_amdgcn_s_waitcnt(0);
          __syncthreads();
          if (ok0) write_back(q0, Wc, Ic, I0);
        } else {
          Wc = ld2(w + p);
          Ic = ld2(inc + p);
          ws = ld2(w + ps);
          is = ld2(inc + ps);
        }
        FSc = ld2(af + g.fS(ic, jc));
        Ws = hs ? ws : zero2;
        Is = hs ? is : zero2;
      }
#pragma unroll 1
      for (int r = 0; r < RPW; ++r) {
        const int j = j0 + r;
        const bool ok = j < n && lane_ok;
        const int jc = ok ? j : 0;
        const int64_t p = (int64_t)jc * n + ic;
        const bool hn = ok && jc < n - 1;
        const int64_t pn = hn ? p + n : p;
        double2 Wl, Il;
        if constexpr (FUSED) {
          if (r + 1 < RPW) {   // an own row: updated, written back, kept as the window's next
            double2 Iold;
            advance(pn, Wl, Il, Iold);
            if (hn) write_back(pn, Wl, Il, Iold);
          } else {
            Wl = Wh;
            Il = Ih;
          }
        } else {
          Wl = ld2(w + pn);
          Il = ld2(inc + pn);
        }
        const float2 Df = *reinterpret_cast<const float2*>(dvf + p);
        const double2 D = make_double2(Df.x, Df.y);
        const double2 FN = ld2(af + g.fN(ic, jc));
        // x-faces i0, i0 + 1, i0 + 2 of the row: the aligned pair is (i0, i0 + 1) on even
        // rows and (i0 + 1, i0 + 2) on odd ones (rows hold n + 1 faces)
        const int64_t fx = g.fW(ic, jc);
        const bool odd = (jc & 1) != 0;
        const double2 A = ld2(af + (odd ? fx + 1 : fx));
        const double as = af[odd ? fx : fx + 2];
        const double a0 = odd ? as : A.x, a1 = odd ? A.x : A.y, a2 = odd ? A.y : as;
        const double2 W = Wc, I = Ic, FS = FSc;
        const double2 Wn = hn ? Wl : zero2, In = hn ? Il : zero2;
        const double wW = dppd<0x138>(W.y), iW = dppd<0x138>(I.y);   // column i0 - 1
        const double wE = dppd<0x130>(W.x), iE = dppd<0x130>(I.x);   // column i0 + 2
        const double dW0 = (W.x - (hw0 ? wW : 0.0)) + (I.x - (hw0 ? iW : 0.0));
        const double dE0 = (W.x - W.y) + (I.x - I.y);
        const double dS0 = (W.x - Ws.x) + (I.x - Is.x);
        const double dN0 = (W.x - Wn.x) + (I.x - In.x);
        const double dW1 = (W.y - W.x) + (I.y - I.x);
        const double dE1 = (W.y - (he1 ? wE : 0.0)) + (I.y - (he1 ? iE : 0.0));
        const double dS1 = (W.y - Ws.y) + (I.y - Is.y);
        const double dN1 = (W.y - Wn.y) + (I.y - In.y);
        const double au0 = a0 * dW0 + a1 * dE0 + FS.x * dS0 + FN.x * dN0;
        const double au1 = a1 * dW1 + a2 * dE1 + FS.y * dS1 + FN.y * dN1;
        const double rv0 = tauf - c * au0 - I.x, rv1 = tauf - c * au1 - I.y;
        // invalid lanes write the spare word pair after the n^2 tile
        *reinterpret_cast<float2*>(xs + (ok ? j * n + i0 : n * n)) =
            make_float2((float)(D.x * rv0), (float)(D.y * rv1));
        if (ok) {
          // a non-finite residual turns bad into NaN (v_max_f64 would drop it)
          bad = fma(rv0, 0.0, fma(rv1, 0.0, bad));
          acc[0] = fmax(acc[0], fmax(fabs(rv0), fabs(rv1)));
          acc[1] = fmax(acc[1], fmax(fabs(W.x + I.x), fabs(W.y + I.y)));
          acc[2] = fmax(acc[2], fmax(D.x * fabs(rv0), D.y * fabs(rv1)));
        }
        Ws = W;
        Is = I;
        Wc = Wl;
        Ic = Il;
        FSc = FN;
      }
      if (bad != bad) acc[0] = bad;
      block_max_nn<NW, 3>(acc, dslots, lane, wave);
      return;
    }
    if constexpr (!FUSED) {   // odd n: updates run in their own passes
#pragma unroll 1
    for (int k0 = 0; k0 < RPW * CPL; k0 += KG) {
      float rhs[KG];
      int64_t pp[KG];
      bool okk[KG];
#pragma unroll
      for (int u = 0; u < KG; ++u) {
        const int k = k0 + u;
        const int j = j0 + k / CPL, i = i0 + k % CPL;
        const bool ok = j < n && i < n;
        // clamped indices keep every load in bounds without a branch, so a group's loads
        // are in flight together; neighbours outside the grid are selected away (0)
        const int ic = ok ? i : 0, jc = ok ? j : 0;
        const int64_t p = (int64_t)jc * n + ic;
        const bool hw = ic > 0, he = ic < n - 1, hs = jc > 0, hn = jc < n - 1;
        const int64_t pw = hw ? p - 1 : p, pe = he ? p + 1 : p;
        const int64_t ps = hs ? p - n : p, pn = hn ? p + n : p;
        const double wp = w[p], ip = inc[p];
        const double ww = w[pw], iw = inc[pw], we = w[pe], ie = inc[pe];
        const double wsv = w[ps], isv = inc[ps], wnv = w[pn], inv = inc[pn];
        // neighbour differences of w and of inc taken separately: forming w + inc first
        // would round at the scale of |w| before the stencil amplifies it
        const double dW = (wp - (hw ? ww : 0.0)) + (ip - (hw ? iw : 0.0));
        const double dE = (wp - (he ? we : 0.0)) + (ip - (he ? ie : 0.0));
        const double dS = (wp - (hs ? wsv : 0.0)) + (ip - (hs ? isv : 0.0));
        const double dN = (wp - (hn ? wnv : 0.0)) + (ip - (hn ? inv : 0.0));
        const double au = af[g.fW(ic, jc)] * dW + af[g.fE(ic, jc)] * dE + af[g.fS(ic, jc)] * dS +
                          af[g.fN(ic, jc)] * dN;
        const double rv = tauf - c * au - ip;
        const double dp = dvf[p];
        rhs[u] = (float)(dp * rv);
        pp[u] = p;
        okk[u] = ok;
        acc[0] = ok ? nanmax(acc[0], fabs(rv)) : acc[0];
        acc[1] = ok ? nanmax(acc[1], fabs(wp + ip)) : acc[1];
        acc[2] = ok ? nanmax(acc[2], dp * fabs(rv)) : acc[2];
      }
#pragma unroll
      for (int u = 0; u < KG; ++u)
        if (okk[u]) xs[pp[u]] = rhs[u];
    }
    }
    block_max_nn<NW, 3>(acc, dslots, lane, wave);
  };

  for (int step = 0; step < J; ++step) {
    // The step is solved for its increment inc = w_{j+1} - w_j, starting from the earlier
    // increments: for a constant source inc_j = R inc_{j-1} with R = (I + tau A)^{-1}, so a
    // mode damped by rho per step leaves (1 - rho) of itself in the guess inc_{j-1} and
    // (1 - rho)^2 in 2 inc_{j-1} - inc_{j-2}; the slowest modes (rho near 1) dominate
    // what is left, and the second guess shrinks them by another factor 1 - rho (zero
    // increment at the first step of a slice, inc_0 at the second).  Each pass recomputes
    // the true float64 residual from w_j and inc; only inc changes during the step.
    double acc[3];
    if (pairs && step > 0)   // closes step j - 1: w_j, and the start 2 inc_{j-1} - inc_{j-2}
      residual(acc, std::integral_constant<int, kSweepStart>{}, step > 1 ? 2.0 : 1.0, step > 1 ? -1.0 : 0.0);
    else
      residual(acc, std::integral_constant<int, kSweepPlain>{}, 0.0, 0.0);
    double rmax = acc[0];
    double sig = acc[2];   // float32 right-hand sides are normalised by their max
    // The rounding allowance scales with the largest |w_j + inc| the step has reached: a
    // slice that starts from a zero state has none at its first sweep, while the
    // recomputed residual of the grown increment cannot fall below its float64 floor.
    double wref = acc[1];
    double target = residual_target(tol, wref, tauf, dmax);
    int pass = 0;
    while (rmax > target && sig > 0.0 && pass < kMaxRefinePasses) {
      // the owner's right-hand side: the residual sweep's tile scaled by 1/sig (late
      // residuals shrink towards the float64 floor and their squares would underflow)
      const float fis = (float)(1.0 / sig);
      if constexpr (!RB) {
        float rr = 0.f;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
          int j = j0 + r;
#pragma unroll
          for (int t = 0; t < CPL; ++t) {
            int i = i0 + t;
            float v = (j < n && i < n) ? xs[j * n + i] * fis : 0.f;
            R[r][t] = v;
            P[r][t] = v;
            X[r][t] = 0.f;
            rr = fmaf(v, v, rr);
          }
        }
        RS::store_halo(R, P, NS, hr_top, hp_top, hr_bot, hp_bot, lane, wave);
        rr = block_sum_f<NW>(rr, fslots[1], lane, wave);
        const float rel = (float)fmin(0.5, fmax((double)pcg_rtol, kPassMargin * target / rmax));
        const float stop = rel * rel * rr;
        float beta = 0.f;
        int it = 0;
        const long long t0 = clock64();
        while (rr > stop && it < maxit) {
          float pq = RS::matvec(P, Q, EW, NS, hr_top, hp_top, hr_bot, hp_bot, beta, lane, wave);
          pq = block_sum_f<NW>(pq, fslots[0], lane, wave);
          // CG scalars through the hardware reciprocal (about 1 ulp): an IEEE division
          // costs some ten instructions per iteration of an issue-bound loop
          const float alpha = rr * __builtin_amdgcn_rcpf(pq);
          float rn = 0.f;
#pragma unroll
          for (int r = 0; r < RPW; ++r)
#pragma unroll
            for (int t = 0; t < CPL; ++t) {
              X[r][t] = fmaf(alpha, P[r][t], X[r][t]);
              R[r][t] = fmaf(-alpha, Q[r][t], R[r][t]);
              rn = fmaf(R[r][t], R[r][t], rn);
            }
          RS::store_halo(R, P, NS, hr_top, hp_top, hr_bot, hp_bot, lane, wave);
          rn = block_sum_f<NW>(rn, fslots[1], lane, wave);
          beta = rn * __builtin_amdgcn_rcpf(rr);
          rr = rn;
#pragma unroll
          for (int r = 0; r < RPW; ++r)
#pragma unroll
            for (int t = 0; t < CPL; ++t) P[r][t] = fmaf(beta, P[r][t], R[r][t]);
          ++it;
        }
        t_cg += clock64() - t0;
        if (it >= maxit && rr > stop) fail = true;
        tot_it += it;
        max_it = it > (int)max_it ? it : max_it;
        // correction of the owned nodes: inc += sig D^{-1/2} X (through the thread's own xs
        // entries, so the float64 loop needs no register copy of X)
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
          int j = j0 + r;
#pragma unroll
          for (int t = 0; t < CPL; ++t) {
            int i = i0 + t;
            if (j < n && i < n) xs[j * n + i] = X[r][t];
          }
        }
      } else {
        const float rel = (float)fmin(0.5, fmax((double)pcg_rtol, kPassMargin * target / rmax));
        const RbPassOut po = rb_pass<NW, RPW>(
            (lds_float*)xs, fis, sfm, n, g.nx, rel, maxit, (lds_float*)hr_top, (lds_float*)hp_top,
            (lds_float*)hr_bot, (lds_float*)hp_bot, (lds_float*)ht_top, (lds_float*)ht_bot,
            (lds_float*)fslots[0], (lds_float*)fslots[1]);
        t_cg += po.cycles;
        if (po.capped) fail = true;
        tot_it += po.it;
        max_it = po.it > (int)max_it ? po.it : max_it;
      }
      if (pairs) {
        // the sweep adds sig D^{-1/2} x to inc row by row; it reads the x of its
        // neighbours' rows, which the pass has just written
        __syncthreads();
        residual(acc, std::integral_constant<int, kSweepCorrect>{}, sig, 0.0);
      } else {
#pragma unroll 1
        for (int k0 = 0; k0 < RPW * CPL; k0 += KU) {
          double v[KU];
          int64_t pp[KU];
          bool okk[KU];
#pragma unroll
          for (int u = 0; u < KU; ++u) {   // branch-free loads (clamped), guarded stores
            const int k = k0 + u;
            const int j = j0 + k / CPL, i = i0 + k % CPL;
            const bool ok = j < n && i < n;
            const int64_t p = ok ? (int64_t)j * n + i : 0;
            v[u] = inc[p] + sig * (double)dvf[p] * (double)xs[p];
            pp[u] = p;
            okk[u] = ok;
          }
#pragma unroll
          for (int u = 0; u < KU; ++u)
            if (okk[u]) inc[pp[u]] = v[u];
        }
        __syncthreads();   // the residual sweep reads neighbours' inc
        residual(acc, std::integral_constant<int, kSweepPlain>{}, 0.0, 0.0);
      }
      rmax = acc[0];
      sig = acc[2];
      wref = fmax(wref, acc[1]);
      target = residual_target(tol, wref, tauf, dmax);
      ++pass;
    }
    tot_pass += pass;
    if (rmax > target) {
      fail = true;
      ++missed;
    }
    // with column pairs the next step's first sweep closes this one
    if (pairs && step + 1 < J) continue;
    // w_{j+1} = w_j + inc, and the next step's starting increment: extrapolated linearly
    // in the increments, 2 inc_j - inc_{j-1} (inc_j itself after the first step of a slice)
    const double ka = step > 0 ? 2.0 : 1.0, kb = step > 0 ? -1.0 : 0.0;
    if (pairs) {
#pragma unroll 1
      for (int r0 = 0; r0 < RPW; r0 += KR) {
        double2 Wv[KR], I[KR], IP[KR];
#pragma unroll
        for (int u = 0; u < KR && r0 + u < RPW; ++u) {
          const int j = j0 + r0 + u;
          const int64_t p = (j < n && i0 < n) ? (int64_t)j * n + i0 : 0;
          Wv[u] = ld2(w + p);
          I[u] = ld2(inc + p);
          IP[u] = ld2(incp + p);
        }
#pragma unroll
        for (int u = 0; u < KR && r0 + u < RPW; ++u) {
          const int j = j0 + r0 + u;
          if (j < n && i0 < n) {
            const int64_t p = (int64_t)j * n + i0;
            st2(w + p, Wv[u].x + I[u].x, Wv[u].y + I[u].y);
            st2(inc + p, ka * I[u].x + kb * IP[u].x, ka * I[u].y + kb * IP[u].y);
            st2(incp + p, I[u].x, I[u].y);
          }
        }
      }
    } else
#pragma unroll 1
    for (int k0 = 0; k0 < RPW * CPL; k0 += KU) {
      double v[KU], ic[KU], ip[KU];
      int64_t pp[KU];
      bool okk[KU];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int k = k0 + u;
        const int j = j0 + k / CPL, i = i0 + k % CPL;
        const bool ok = j < n && i < n;
        const int64_t p = ok ? (int64_t)j * n + i : 0;
        ic[u] = inc[p];
        ip[u] = incp[p];
        v[u] = w[p] + ic[u];
        pp[u] = p;
        okk[u] = ok;
      }
#pragma unroll
      for (int u = 0; u < KU; ++u)
        if (okk[u]) {
          w[pp[u]] = v[u];
          inc[pp[u]] = ka * ic[u] + kb * ip[u];
          incp[pp[u]] = ic[u];
        }
    }
    __syncthreads();   // the next residual sweep reads neighbours' w and inc
  }
  tally.its += tot_it;
  tally.passes += tot_pass;
  tally.steps += (unsigned long long)J;
  tally.max_it = max_it > tally.max_it ? max_it : tally.max_it;
  tally.missed += missed;
  tally.cg_cycles += t_cg;
  tally.fail = tally.fail || fail;
}

// One work-group per (sample, slice) system of an [M][N] batch.
template <int NW, int CPL, int RPW, bool RB = false>
__global__ __launch_bounds__(64 * NW) void fine2d_resident_kernel(
    const double* __restrict__ a, const float* __restrict__ sf, const double* __restrict__ dinv,
    const float* __restrict__ dinvf,
    int n, double c, double tauf, int J, double tol, float pcg_rtol, int maxit, StartRef sr,
    double* __restrict__ out, double* __restrict__ incbuf, int64_t M, int N, int skip_first, const uint8_t* __restrict__ active, int* __restrict__ flag,
    unsigned long long* __restrict__ cnt) {
  const long long t_start = clock64();
  // the slices of a sample share its coefficients (and scaled forms): XCD-major order
  // keeps them under one L2
  const int64_t sys = xcd_major(blockIdx.x, gridDim.x);
  const int64_t m = sys / N;
  const int s = (int)(sys % N);
  if (active && !active[m]) return;
  if (skip_first && s == 0) return;
  const int64_t Nx = (int64_t)n * n;
  ResTally tl;
  // increments of the current and the previous step in [2][nsys][Nx]
  resident_system<NW, CPL, RPW, RB>(a, sf, dinv, dinvf, n, c, tauf, J, tol, pcg_rtol, maxit,
                                    sr.row(m, s, N, Nx), out + sys * Nx, incbuf + sys * Nx,
                                    incbuf + ((int64_t)gridDim.x + sys) * Nx, m, tl);
  report_tally(tl, t_start, flag, cnt);
}

template <int NW, int CPL, int RPW, bool RB = false>
void launch_resident(hipStream_t st, int64_t nsys, const double* a, const float* sf,
                     const double* dinv, const float* dinvf, int n, double c, double tauf, int J, double tol,
                     float pcg_rtol, int maxit, StartRef sr, double* out, double* incbuf, int64_t M, int N,
                     int skip_first, const uint8_t* active, int* flag, unsigned long long* cnt) {
  size_t lds = sizeof(float) * ((size_t)n * n + 2);   // n^2 tile + a spare word pair
  fine2d_resident_kernel<NW, CPL, RPW, RB><<<dim3((unsigned)nsys), dim3(64 * NW), lds, st>>>(
      a, sf, dinv, dinvf, n, c, tauf, J, tol, pcg_rtol, maxit, sr, out, incbuf, M, N, skip_first, active,
      flag, cnt);
  KC_LAUNCH_CHECK();
}

// One class of a ragged batch as the persistent fine launch reads it (device copy).
struct PersistClass {
  const double* a;          // [M][Fc] faces
  const float* sf;          // [M][Fc] scaled float32 couplings
  const double* dinv;       // [M][Nx] D^{-1/2}
  const float* dinvf;       // [M][Nx] its float32 copy
  const double* U;          // starts in the parareal layout (slice s from U[m][s-1])
  const double* u0;         // slice 0's start (nullable: zero)
  const uint8_t* active;    // [M] nullable
  double* out;              // [M][N][Nx]
  double c, tauf, tol;
  int64_t first;            // index of the class's first task
  int n, N, J, maxit;
  float pcg_rtol;
};

// The fine sweeps of several classes (grids up to 128 x 128, any N and J) in one launch:
// every work-group takes (class, sample, slice) tasks from device counters until none is
// left, and solves each as fine2d_resident_kernel solves its system (same code, so the same
// result bit for bit).  Tasks are numbered class by class, sample-major, and dealt to the
// XCDs in eight contiguous ranges, one counter each: a work-group takes from its own XCD's
// range first (the slices of a sample share their coefficients under one L2), then from the
// others.  Every work-group leaves once all eight counters have passed their range, so the
// launch ends whatever the timing.  Retired samples' tasks are skipped.  incbuf: two rows of
// nx_max per work-group; queue: 8 counters, zero at launch.
template <int NW, int CPL, int RPW, bool RB>
__global__ __launch_bounds__(64 * NW) void fine2d_persistent_kernel(
    const PersistClass* __restrict__ cls, int ncls, int64_t ntasks, int skip_first,
    double* __restrict__ incbuf, int64_t nx_max, unsigned long long* __restrict__ queue,
    int* __restrict__ flag, unsigned long long* __restrict__ cnt) {
  const long long t_start = clock64();
  __shared__ long long task_s;
  ResTally tl;
  double* inc = incbuf + 2 * (int64_t)blockIdx.x * nx_max;
  double* incp = inc + nx_max;
  const int home = (int)(blockIdx.x % kXcds);
  int tried = 0;   // thread 0: ranges found empty
  for (;;) {
    if (threadIdx.x == 0) {
      long long t = -1;
      while (tried < kXcds) {
        const int x = (home + tried) % kXcds;
        const int64_t lo = ntasks * x / kXcds, hi = ntasks * (x + 1) / kXcds;
        const unsigned long long k = atomicAdd(&queue[x], 1ull);
        if ((int64_t)k < hi - lo) {
          t = lo + (int64_t)k;
          break;
        }
        ++tried;
      }
      task_s = t;
    }
    __syncthreads();
    const long long tv = task_s;
    __syncthreads();   // read by all before thread 0 writes the next task
    const long long t = ((long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(tv >> 32)) << 32) |
                        (unsigned)__builtin_amdgcn_readfirstlane((int)tv);
    if (t < 0) break;
    int k = 0;
    while (k + 1 < ncls && t >= cls[k + 1].first) ++k;
    const PersistClass& C = cls[k];
    const int64_t local = t - C.first;
    const int64_t m = local / C.N;
    const int s = (int)(local % C.N);
    if (C.active && !C.active[m]) continue;
    if (skip_first && s == 0) continue;
    const int64_t Nx = (int64_t)C.n * C.n;
    const StartRef sr{C.U, C.u0, true};
    resident_system<NW, CPL, RPW, RB>(C.a, C.sf, C.dinv, C.dinvf, C.n, C.c, C.tauf, C.J, C.tol, C.pcg_rtol,
                                      C.maxit, sr.row(m, s, C.N, Nx), C.out + local * Nx, inc, incp, m, tl);
  }
  report_tally(tl, t_start, flag, cnt);
}

__global__ void queue_reset_kernel(unsigned long long* q) {
  if (threadIdx.x < kXcds) q[threadIdx.x] = 0ull;
}

}  // namespace

// 2D system tables (float64 D^{-1/2} and float32 scaled coefficients) for tau.
void build_tables_2d(hipStream_t st, const double* a, int n, double c, int64_t M, double* dinv, float* dinvf,
                     float* sf) {
  int64_t Nx = (int64_t)n * n;
  dim3 b(256);
  dinv_kernel<<<dim3((unsigned)((Nx + 255) / 256), (unsigned)M), b, 0, st>>>(a, n, c, M, dinv, dinvf);
  KC_LAUNCH_CHECK();
  if (sf) {
    int64_t Fc = 2LL * n * (n + 1);
    scaled_faces_kernel<<<dim3((unsigned)((Fc + 255) / 256), (unsigned)M), b, 0, st>>>(a, dinv, n, c,
                                                                                        M, sf);
    KC_LAUNCH_CHECK();
  }
}

// Generic driver: J steps of size tau on every (m, s) of an [M][N] batch.
int propagate_impl(klecgc_ctx* ctx, const klecgc_problem& p, const FineArgs& fa, double tau, int J,
                   int N) {
  hipStream_t st = ctx->stream;
  const int n = p.n;
  const double h = 1.0 / (n + 1);
  const double c = tau / (h * h);
  const double tauf = tau * p.forcing;
  const int64_t M = fa.M;
  const int64_t nsys = M * N;
  StartRef sr{fa.start, fa.u0, fa.start_shift};
  DevStatus ds = status_block(ctx);
  status_reset(ctx, ds);
  int* flag = ds.flag;
  unsigned long long* cnt = ds.cnt;
  if (p.dim == 1) {
    double* tab = (double*)ctx->ws.get(WS_FACTORS, sizeof(double) * 3 * n * M);
    tri_factor_kernel<<<dim3((unsigned)((M + 63) / 64)), dim3(64), 0, st>>>(fa.a, n, c, M, tab);
    KC_LAUNCH_CHECK();
    timed(ctx, KT_FINE, [&] {
      fine1d_kernel<<<dim3((unsigned)((nsys + 63) / 64)), dim3(64), 0, st>>>(
          tab, n, J, tauf, sr, fa.out, M, N, fa.skip_first, fa.active);
      KC_LAUNCH_CHECK();
    });
    return KC_OK;
  }
  const int64_t Nx = (int64_t)n * n;
  const int64_t Fc = 2LL * n * (n + 1);
  const double tol = p.inner_rtol > 0 ? p.inner_rtol : 1e-13;
  const int maxit = p.inner_max_iter > 0 ? p.inner_max_iter : 4000;
  // float64 D^{-1/2} [M][Nx], then its float32 copy [M][Nx] (the resident kernels scale the
  // float32 right-hand sides and corrections with it: a consistent scaling, not an accuracy
  // question, since the float64 residuals alone decide convergence)
  double* dinv = (double*)ctx->ws.get(WS_DINV, (sizeof(double) + sizeof(float)) * Nx * M);
  float* dinvf = (float*)(dinv + Nx * M);
  const KcTuning tu = tuning_for(ctx, n);
  const int variant = p.precision == KC_PREC_F32_REFINED ? fine_variant_for(n, tu.fine_variant) : KC_FINE_STREAM64;
  const bool resident = variant != KC_FINE_STREAM64 && variant != KC_FINE_MG;
  const bool scaled = variant != KC_FINE_STREAM64;
  float* sf = scaled ? (float*)ctx->ws.get(WS_FSCALED, sizeof(float) * Fc * M) : nullptr;
  build_tables_2d(st, fa.a, n, c, M, dinv, dinvf, sf);
  // increments of the current and the previous step per system ([2][nsys][Nx])
  double* incbuf = resident ? (double*)ctx->ws.get(WS_FINE_INC, 2 * sizeof(double) * Nx * nsys) : nullptr;
  double* scr = variant == KC_FINE_STREAM64 ? (double*)ctx->ws.get(WS_KRYLOV, sizeof(double) * 3 * Nx * nsys)
                                            : nullptr;
  const float pcg_rtol = tu.fine_pcg_rtol;
  timed(ctx, KT_FINE, [&] {
    switch (variant) {
      case KC_FINE_RES16:
        launch_resident<8, 1, 2>(st, nsys, fa.a, sf, dinv, dinvf, n, c, tauf, J, tol, pcg_rtol, maxit, sr, fa.out, incbuf,
                                 M, N, fa.skip_first, fa.active, flag, cnt);
        break;
      case KC_FINE_RES32:
        launch_resident<8, 1, 4>(st, nsys, fa.a, sf, dinv, dinvf, n, c, tauf, J, tol, pcg_rtol, maxit, sr, fa.out, incbuf,
                                 M, N, fa.skip_first, fa.active, flag, cnt);
        break;
      case KC_FINE_RES64:
        launch_resident<8, 1, 8>(st, nsys, fa.a, sf, dinv, dinvf, n, c, tauf, J, tol, pcg_rtol, maxit, sr, fa.out, incbuf,
                                 M, N, fa.skip_first, fa.active, flag, cnt);
        break;
      case KC_FINE_RES128:
        launch_resident<KC_RES128_NW, 2, 128 / KC_RES128_NW>(st, nsys, fa.a, sf, dinv, dinvf, n, c, tauf, J, tol, pcg_rtol,
                                                             maxit, sr, fa.out, incbuf, M, N, fa.skip_first,
                                                             fa.active, flag, cnt);
        break;
      case KC_FINE_RB128:
        launch_resident<KC_RES128_NW, 2, 128 / KC_RES128_NW, true>(st, nsys, fa.a, sf, dinv, dinvf, n, c, tauf, J, tol, pcg_rtol,
                                                             maxit, sr, fa.out, incbuf, M, N, fa.skip_first,
                                                             fa.active, flag, cnt);
        break;
      case KC_FINE_MG: {
        const int r = fine_mg_streamed(ctx, p, fa, tau, J, N, dinv, sf, flag, cnt);
        if (r != KC_OK) throw Error{r, "multigrid fine propagation failed"};
        break;
      }
      default:
        fine2d_pcg64_kernel<<<dim3((unsigned)nsys), dim3(kStreamThreads), 0, st>>>(
            fa.a, dinv, n, c, tauf, J, tol, maxit, sr, fa.out, scr, M, N, fa.skip_first, fa.active, flag, cnt);
        KC_LAUNCH_CHECK();
    }
  });
  return status_collect(ctx, ds, 0) ? KC_ENOCONV : KC_OK;
}

bool fine_variant_fits(int v, int n) {
  switch (v) {
    case KC_FINE_STREAM64: return true;
    case KC_FINE_RES16: return n <= 16;
    case KC_FINE_RES32: return n <= 32;
    case KC_FINE_RES64: return n <= 64;
    case KC_FINE_RES128: return n <= 128;
    case KC_FINE_RB128: return n <= 128;
    case KC_FINE_MG: return true;
    default: return false;
  }
}

int fine_variant_for(int n, int requested) {
  if (requested >= 0 && fine_variant_fits(requested, n)) return requested;
  if (n <= 16) return KC_FINE_RES16;
  if (n <= 32) return KC_FINE_RES32;
  if (n <= 64) return KC_FINE_RES64;
  if (n <= 128) return KC_FINE_RB128;
  return KC_FINE_MG;
}

bool persistent_eligible(const klecgc_problem& p) {
  return p.dim == 2 && p.precision == KC_PREC_F32_REFINED && p.n <= 128;
}

PersistPlan persistent_prepare(klecgc_ctx* ctx, const std::vector<PersistSpec>& specs) {
  PersistPlan pl;
  hipStream_t st = ctx->stream;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  size_t bytes = al(sizeof(PersistClass) * specs.size()) + al(sizeof(unsigned long long) * kXcds);
  for (const PersistSpec& sp : specs) {
    KC_REQUIRE(persistent_eligible(sp.p), KC_EINVAL, "persistent fine launch: 2D float32-refined classes, n <= 128");
    const int64_t Nx = (int64_t)sp.p.n * sp.p.n, Fc = 2LL * sp.p.n * (sp.p.n + 1);
    bytes += al(sizeof(double) * sp.M * Nx) + al(sizeof(float) * sp.M * Nx) + al(sizeof(float) * sp.M * Fc);
  }
  char* base = (char*)ctx->ws.get(WS_PERSIST, bytes);
  char* q = base;
  pl.cls = q;
  q += al(sizeof(PersistClass) * specs.size());
  pl.queue = (unsigned long long*)q;
  q += al(sizeof(unsigned long long) * kXcds);
  std::vector<PersistClass> h(specs.size());
  int64_t first = 0;
  for (size_t i = 0; i < specs.size(); ++i) {
    const PersistSpec& sp = specs[i];
    const int n = sp.p.n;
    const int64_t Nx = (int64_t)n * n, Fc = 2LL * n * (n + 1);
    double* dinv = (double*)q;
    q += al(sizeof(double) * sp.M * Nx);
    float* dinvf = (float*)q;
    q += al(sizeof(float) * sp.M * Nx);
    float* sf = (float*)q;
    q += al(sizeof(float) * sp.M * Fc);
    // the same step, tables and stopping rule as propagate_impl
    const double tau = sp.p.T / sp.p.N / sp.p.J;
    const double hh = 1.0 / (n + 1);
    const double c = tau / (hh * hh);
    build_tables_2d(st, sp.a, n, c, sp.M, dinv, dinvf, sf);
    PersistClass& d = h[i];
    d.a = sp.a;
    d.sf = sf;
    d.dinv = dinv;
    d.dinvf = dinvf;
    d.U = sp.U;
    d.u0 = sp.u0;
    d.active = sp.active;
    d.out = sp.out;
    d.c = c;
    d.tauf = tau * sp.p.forcing;
    d.tol = sp.p.inner_rtol > 0 ? sp.p.inner_rtol : 1e-13;
    d.first = first;
    d.n = n;
    d.N = sp.p.N;
    d.J = sp.p.J;
    d.maxit = sp.p.inner_max_iter > 0 ? sp.p.inner_max_iter : 4000;
    d.pcg_rtol = sp.pcg_rtol;
    first += sp.M * sp.p.N;
    pl.nmax = std::max(pl.nmax, n);
  }
  KC_TRY_HIP(hipMemcpyAsync(pl.cls, h.data(), sizeof(PersistClass) * h.size(), hipMemcpyHostToDevice, st));
  KC_TRY_HIP(hipStreamSynchronize(st));   // h is a host temporary
  pl.ncls = (int)specs.size();
  pl.ntasks = first;
  pl.grid = std::max(ctx->num_cus, kXcds);
  pl.incbuf = (double*)ctx->ws.get(WS_FINE_INC, 2 * sizeof(double) * (size_t)pl.grid * pl.nmax * pl.nmax);
  return pl;
}

void persistent_launch(klecgc_ctx* ctx, hipStream_t st, const PersistPlan& pl, int skip_first) {
  if (pl.ntasks == 0) return;
  DevStatus ds = status_block(ctx);
  queue_reset_kernel<<<1, 64, 0, st>>>(pl.queue);
  KC_LAUNCH_CHECK();
  const size_t lds = sizeof(float) * ((size_t)pl.nmax * pl.nmax + 2);
  auto go = [&] {
    fine2d_persistent_kernel<KC_RES128_NW, 2, 128 / KC_RES128_NW, true>
        <<<dim3((unsigned)pl.grid), dim3(64 * KC_RES128_NW), lds, st>>>(
            (const PersistClass*)pl.cls, pl.ncls, pl.ntasks, skip_first, pl.incbuf, (int64_t)pl.nmax * pl.nmax,
            pl.queue, ds.flag, ds.cnt);
    KC_LAUNCH_CHECK();
  };
  if (st == ctx->stream)
    timed(ctx, KT_FINE, go);
  else
    go();
}

int fine_propagate_impl(klecgc_ctx* ctx, const klecgc_problem& p, const FineArgs& fa) {
  return propagate_impl(ctx, p, fa, p.T / p.N / p.J, p.J, p.N);
}

// Sequential sweep over the slices: U[m][s] = P(U[m][s-1]) with P = J steps of tau,
// each launch advancing all samples by one slice (an [M][1] batch).
static int sweep_impl(klecgc_ctx* ctx, const klecgc_problem& p, const double* a, const double* u0,
                      int64_t M, double* U, double tau, int J) {
  const int64_t Nx = n_unknowns(p);
  int rc = KC_OK;
  double* stage = (double*)ctx->ws.get(WS_START, sizeof(double) * Nx * M);
  double* outb = (double*)ctx->ws.get(WS_GEMM_A, sizeof(double) * Nx * M);
  for (int s = 0; s < p.N; ++s) {
    if (s == 0) {
      if (u0)
        KC_TRY_HIP(hipMemcpyAsync(stage, u0, sizeof(double) * Nx * M, hipMemcpyDeviceToDevice, ctx->stream));
      else
        KC_TRY_HIP(hipMemsetAsync(stage, 0, sizeof(double) * Nx * M, ctx->stream));
    } else {
      KC_TRY_HIP(hipMemcpy2DAsync(stage, sizeof(double) * Nx, U + (s - 1) * Nx, sizeof(double) * Nx * p.N,
                                  sizeof(double) * Nx, M, hipMemcpyDeviceToDevice, ctx->stream));
    }
    FineArgs fa{a, stage, nullptr, false, 0, nullptr, outb, M};
    int r = propagate_impl(ctx, p, fa, tau, J, 1);
    if (r != KC_OK) rc = r;
    KC_TRY_HIP(hipMemcpy2DAsync(U + s * Nx, sizeof(double) * Nx * p.N, outb, sizeof(double) * Nx,
                                sizeof(double) * Nx, M, hipMemcpyDeviceToDevice, ctx->stream));
  }
  return rc;
}

int coarse_sweep_impl(klecgc_ctx* ctx, const klecgc_problem& p, const double* a, const double* u0,
                      int64_t M, double* U) {
  return sweep_impl(ctx, p, a, u0, M, U, p.T / p.N, 1);
}

int serial_fine_impl(klecgc_ctx* ctx, const klecgc_problem& p, const double* a, const double* u0,
                     int64_t M, double* U) {
  return sweep_impl(ctx, p, a, u0, M, U, p.T / p.N / p.J, p.J);
}

}  // namespace kc
