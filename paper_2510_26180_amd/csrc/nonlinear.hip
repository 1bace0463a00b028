// The nonlinear examples of Sections 5.2 (Burgers) and 5.3 (Allen-Cahn) on the GPU, with the
// Newton form of the diagonalised coarse grid correction (Section 3.2, eq. Newton2 with the
// averaged Jacobian of eq. Jac).
//
// Both problems are 1D with tridiagonal Jacobians, at most a few hundred unknowns per state.
// Every tridiagonal system -- the Newton steps of each backward-Euler step of F and G, and the
// shifted systems (lambda_k I - dT Jbar) q_k = p_k of step (b) -- is solved by one work-group
// holding the system in LDS, one row per thread, by parallel cyclic reduction (log2 P
// reduction steps, P the power of two at or above n), so that a batch of thousands of
// (sample, slice) systems keeps many independent work-groups per CU.  A backward-Euler step
// runs its whole Newton iteration inside the work-group; the convergence test is a block
// reduction, so every thread takes the same decision.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "models.h"
#include "reduce.h"

namespace kc {

namespace {

struct NLP {
  int model;        // KC_MODEL_BURGERS or KC_MODEL_ALLEN_CAHN
  int n;
  double h;
  double left, right;   // Dirichlet values
};

__host__ __device__ inline NLP nl_params(int model, int n) {
  NLP p;
  p.model = model;
  p.n = n;
  if (model == KC_MODEL_BURGERS) {
    p.h = 1.0 / (n + 1);
    p.left = 0.0;
    p.right = 0.0;
  } else {
    p.h = 2.0 / (n + 1);
    p.left = -1.0;
    p.right = 1.0;
  }
  return p;
}

// f_i and row i of grad f at (um, u, up) = (u_{i-1}, u_i, u_{i+1}); c = eps of the sample
__device__ __forceinline__ void f_row(const NLP& P, double c, double um, double u, double up, double& f, double& jl,
                                      double& jd, double& ju) {
  const double ih2 = 1.0 / (P.h * P.h);
  const double lap = (up - 2.0 * u + um) * ih2;
  if (P.model == KC_MODEL_BURGERS) {
    const double nu = c / 50.0;
    const double ih = 1.0 / P.h;
    if (u >= 0.0) {
      f = nu * lap - u * (u - um) * ih;
      jl = nu * ih2 + u * ih;
      jd = -2.0 * nu * ih2 - (2.0 * u - um) * ih;
      ju = nu * ih2;
    } else {
      f = nu * lap - u * (up - u) * ih;
      jl = nu * ih2;
      jd = -2.0 * nu * ih2 - (up - 2.0 * u) * ih;
      ju = nu * ih2 - u * ih;
    }
  } else {
    f = c * lap - (u * u * u - u);
    jl = c * ih2;
    jd = -2.0 * c * ih2 - (3.0 * u * u - 1.0);
    ju = c * ih2;
  }
}

// 1/b from the hardware reciprocal estimate and two Newton-Raphson steps (e = 1 - b r,
// r += r e); the estimate is good to ~5e-8, so two steps reach the last bit (correctly rounded
// on a million random operands over [1e-3, 1e3] on gfx950).  Several times cheaper than the
// IEEE division sequence.
__device__ __forceinline__ double rcp64(double b) {
  double r = __builtin_amdgcn_rcp(b);
  double e = fma(-b, r, 1.0);
  r = fma(r, e, r);
  e = fma(-b, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return cplx{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  const double d = rcp64(b.re * b.re + b.im * b.im);
  return cplx{(a.re * b.re + a.im * b.im) * d, (a.im * b.re - a.re * b.im) * d};
}
__device__ __forceinline__ cplx cneg(cplx a) { return cplx{-a.re, -a.im}; }

struct RealOps {
  using T = double;
  static __device__ __forceinline__ T zero() { return 0.0; }
  static __device__ __forceinline__ T one() { return 1.0; }
  static __device__ __forceinline__ T mul(T a, T b) { return a * b; }
  static __device__ __forceinline__ T add(T a, T b) { return a + b; }
  static __device__ __forceinline__ T div(T a, T b) { return a * rcp64(b); }
  static __device__ __forceinline__ T neg(T a) { return -a; }
};
struct CplxOps {
  using T = cplx;
  static __device__ __forceinline__ T zero() { return cplx{0.0, 0.0}; }
  static __device__ __forceinline__ T one() { return cplx{1.0, 0.0}; }
  static __device__ __forceinline__ T mul(T a, T b) { return cmul(a, b); }
  static __device__ __forceinline__ T add(T a, T b) { return cadd(a, b); }
  static __device__ __forceinline__ T div(T a, T b) { return cdiv(a, b); }
  static __device__ __forceinline__ T neg(T a) { return cneg(a); }
};

// Parallel cyclic reduction of the tridiagonal system whose row i (thread i, i < P = blockDim)
// is (a, b, c | d); rows past the system are identity rows.  lds: 8 P values of T (two
// buffers of a, b, c, d).  Returns x_i.  Starts and ends with a barrier.
template <class O>
__device__ typename O::T pcr_solve(typename O::T a, typename O::T b, typename O::T c, typename O::T d,
                                   typename O::T* lds) {
  using T = typename O::T;
  const int P = blockDim.x, i = threadIdx.x;
  T* buf[2] = {lds, lds + 4 * P};
  __syncthreads();
  buf[0][i] = a;
  buf[0][P + i] = b;
  buf[0][2 * P + i] = c;
  buf[0][3 * P + i] = d;
  int cur = 0;
  __syncthreads();
  for (int s = 1; s < P; s <<= 1) {
    const T* A = buf[cur];
    T* B = buf[cur ^ 1];
    const T ai = A[i], bi = A[P + i], ci = A[2 * P + i], di = A[3 * P + i];
    T am = O::zero(), bm = O::one(), cm = O::zero(), dm = O::zero();
    T ap = O::zero(), bp = O::one(), cp = O::zero(), dp = O::zero();
    if (i >= s) {
      am = A[i - s];
      bm = A[P + i - s];
      cm = A[2 * P + i - s];
      dm = A[3 * P + i - s];
    }
    if (i + s < P) {
      ap = A[i + s];
      bp = A[P + i + s];
      cp = A[2 * P + i + s];
      dp = A[3 * P + i + s];
    }
    const T al = O::neg(O::div(ai, bm));
    const T ga = O::neg(O::div(ci, bp));
    B[i] = O::mul(al, am);
    B[P + i] = O::add(bi, O::add(O::mul(al, cm), O::mul(ga, ap)));
    B[2 * P + i] = O::mul(ga, cp);
    B[3 * P + i] = O::add(di, O::add(O::mul(al, dm), O::mul(ga, dp)));
    cur ^= 1;
    __syncthreads();
  }
  return O::div(buf[cur][3 * P + i], buf[cur][P + i]);
}

// block maxima of two non-negative values (NaN wins); every thread gets both
__device__ __forceinline__ void block_max2(double& x, double& y, double* red) {
  double v[2] = {x, y};
  const bool mx[2] = {true, true};
  block_reduce<2>(v, mx, red);
  x = v[0];
  y = v[1];
}

// One work-group per (listed sample, slice s_lo + k): J backward-Euler steps of size tau, each
// w - tau f(w) = v solved by Newton from w = v until |dw|_inf <= ntol max(|w|_inf, 1).
// Start: mode 0 base[m][s]; 1 (s == 0 ? u0[m] : base[m][s-1]); 2 (s == 0 ? alpha base[m][N-1] :
// base[m][s-1]).  A Newton iteration that reaches nmax keeps its last iterate; fail[m] marks the
// sample and counts[2] counts such steps.
__global__ __launch_bounds__(1024) void nl_sweep_kernel(int model, int n, const double* __restrict__ coef,
                                                        const int32_t* __restrict__ list,
                                                        const double* __restrict__ base,
                                                        const double* __restrict__ u0, int mode, double alpha,
                                                        int s_lo, int nsl, int N, int J, double tau, double ntol,
                                                        int nmax, double* __restrict__ out,
                                                        unsigned int* __restrict__ fail,
                                                        unsigned long long* __restrict__ counts) {
  extern __shared__ double smem[];
  const int P = blockDim.x, i = threadIdx.x;
  double* w = smem;                 // [P]
  double* pcr = smem + P;           // [8 P]
  double* red = smem + 9 * P;       // [32]
  const int64_t li = blockIdx.x / nsl;
  const int s = s_lo + (int)(blockIdx.x % nsl);
  const int64_t m = list ? list[li] : li;
  const NLP Pm = nl_params(model, n);
  const double c = coef[m];
  const double* src;
  double scale = 1.0;
  if (mode == 0) {
    src = base + (m * N + s) * n;
  } else if (s > 0) {
    src = base + (m * N + s - 1) * n;
  } else if (mode == 1) {
    src = u0 + m * n;
  } else {
    src = base + (m * N + N - 1) * n;
    scale = alpha;
  }
  double u = (i < n) ? scale * src[i] : 0.0;
  w[i] = u;
  bool failed = false;
  unsigned long long newton = 0, capped = 0;
  for (int j = 0; j < J; ++j) {
    const double v = u;
    bool done = false;
    for (int it = 0; it < nmax && !done; ++it) {
      ++newton;
      __syncthreads();
      double a = 0.0, b = 1.0, cc = 0.0, d = 0.0;
      if (i < n) {
        const double um = i > 0 ? w[i - 1] : Pm.left;
        const double up = i < n - 1 ? w[i + 1] : Pm.right;
        double f, jl, jd, ju;
        f_row(Pm, c, um, u, up, f, jl, jd, ju);
        a = i > 0 ? -tau * jl : 0.0;
        b = 1.0 - tau * jd;
        cc = i < n - 1 ? -tau * ju : 0.0;
        d = -(u - tau * f - v);
      }
      const double du = pcr_solve<RealOps>(a, b, cc, d, pcr);
      if (i < n) {
        u += du;
        w[i] = u;
      }
      double dmax = i < n ? fabs(du) : 0.0, umax = i < n ? fabs(u) : 0.0;
      block_max2(dmax, umax, red);
      done = dmax <= ntol * fmax(umax, 1.0);
    }
    failed |= !done;
    capped += done ? 0 : 1;
  }
  if (i < n) out[(m * N + s) * n + i] = u;
  if (i == 0) {
    if (failed) atomicOr(&fail[m], 1u);
    atomicAdd(&counts[0], newton);
    atomicAdd(&counts[1], (unsigned long long)J);
    if (capped) atomicAdd(&counts[2], capped);
  }
}

// Averaged Jacobian of eq. Jac: jbar[m][r][i], r = 0 lower, 1 diagonal, 2 upper, the mean over
// the slices of grad f(U_s - b_s), b = Fv - Gv.
__global__ void nl_avgjac_kernel(int model, int n, const double* __restrict__ coef, const int32_t* __restrict__ list,
                                 int N, const double* __restrict__ U, const double* __restrict__ Fv,
                                 const double* __restrict__ Gv, double* __restrict__ jbar) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t m = list ? list[blockIdx.y] : blockIdx.y;
  const NLP Pm = nl_params(model, n);
  const double c = coef[m];
  double sl = 0.0, sd = 0.0, su = 0.0;
  for (int s = 0; s < N; ++s) {
    const int64_t o = (m * N + s) * n;
    const double u = U[o + i] - (Fv[o + i] - Gv[o + i]);
    const double um = i > 0 ? U[o + i - 1] - (Fv[o + i - 1] - Gv[o + i - 1]) : Pm.left;
    const double up = i < n - 1 ? U[o + i + 1] - (Fv[o + i + 1] - Gv[o + i + 1]) : Pm.right;
    double f, jl, jd, ju;
    f_row(Pm, c, um, u, up, f, jl, jd, ju);
    sl += jl;
    sd += jd;
    su += ju;
  }
  const double inv = 1.0 / N;
  jbar[(m * 3 + 0) * n + i] = sl * inv;
  jbar[(m * 3 + 1) * n + i] = sd * inv;
  jbar[(m * 3 + 2) * n + i] = su * inv;
}

// Newton right-hand side in correction form: D = -[(C_alpha (x) I) u - dT Ft(u) - b], row s
// U_s - z_s - dT f(U_s - b_s) - b_s, z_0 = alpha U_{N-1}, z_s = U_{s-1}.
__global__ void nl_newton_rhs_kernel(int model, int n, const double* __restrict__ coef,
                                     const int32_t* __restrict__ list, int N, double alpha, double dT,
                                     const double* __restrict__ U, const double* __restrict__ Fv,
                                     const double* __restrict__ Gv, double* __restrict__ D) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = blockIdx.y;
  const int64_t m = list ? list[blockIdx.z] : blockIdx.z;
  const NLP Pm = nl_params(model, n);
  const double c = coef[m];
  const int64_t o = (m * N + s) * n;
  const double b = Fv[o + i] - Gv[o + i];
  const double u = U[o + i] - b;
  const double um = i > 0 ? U[o + i - 1] - (Fv[o + i - 1] - Gv[o + i - 1]) : Pm.left;
  const double up = i < n - 1 ? U[o + i + 1] - (Fv[o + i + 1] - Gv[o + i + 1]) : Pm.right;
  double f, jl, jd, ju;
  f_row(Pm, c, um, u, up, f, jl, jd, ju);
  const double z = s == 0 ? alpha * U[(m * N + N - 1) * n + i] : U[o - n + i];
  D[o + i] = -(U[o + i] - z - dT * f - b);
}

// (lambda_k I - dT Jbar) q = p for (listed sample, bin k), in place in spec [M][K][n]
__global__ __launch_bounds__(1024) void nl_shift_solve_kernel(int n, const int32_t* __restrict__ list, int K, int N,
                                                              double aroot, double dT,
                                                              const double* __restrict__ jbar,
                                                              cplx* __restrict__ spec) {
  extern __shared__ cplx csm[];
  const int i = threadIdx.x;
  const int64_t li = blockIdx.x / K;
  const int k = blockIdx.x % K;
  const int64_t m = list ? list[li] : li;
  const double th = 2.0 * M_PI * (double)k / (double)N;
  const cplx lam = cplx{1.0 - aroot * cos(th), aroot * sin(th)};
  cplx a = cplx{0.0, 0.0}, b = cplx{1.0, 0.0}, c = cplx{0.0, 0.0}, d = cplx{0.0, 0.0};
  cplx* q = spec + ((size_t)m * K + k) * n;
  if (i < n) {
    const double* J = jbar + (size_t)m * 3 * n;
    a = cplx{i > 0 ? -dT * J[i] : 0.0, 0.0};
    b = cplx{lam.re - dT * J[n + i], lam.im};
    c = cplx{i < n - 1 ? -dT * J[2 * n + i] : 0.0, 0.0};
    d = q[i];
  }
  const cplx x = pcr_solve<CplxOps>(a, b, c, d, csm);
  if (i < n) q[i] = x;
}

__global__ void nl_u0_kernel(int model, int n, int64_t M, double* __restrict__ u0) {
  const NLP P = nl_params(model, n);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < M * n; t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % n);
    if (model == KC_MODEL_BURGERS) {
      u0[t] = sinpi((double)(i + 1) * P.h);
    } else {
      const double x = -1.0 + (double)(i + 1) * P.h;
      u0[t] = 0.53 * x + 0.47 * sinpi(-1.5 * x);
    }
  }
}

// copy of the listed samples' states
__global__ void nl_copy_kernel(const int32_t* __restrict__ list, int64_t nlist, int64_t S,
                               const double* __restrict__ src, double* __restrict__ dst) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nlist * S; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = list[t / S];
    const int64_t o = m * S + t % S;
    dst[o] = src[o];
  }
}

// maxima[2m] = max |U - Uold|, maxima[2m+1] = max |U| over the sample's states
__global__ __launch_bounds__(256) void nl_increment_kernel(const int32_t* __restrict__ list, int64_t S,
                                                           const double* __restrict__ U,
                                                           const double* __restrict__ Uold,
                                                           unsigned long long* __restrict__ maxima) {
  __shared__ double red[8];
  const int64_t m = list[blockIdx.y];
  double inc = 0.0, un = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < S; p += (int64_t)gridDim.x * blockDim.x) {
    const double v = U[m * S + p];
    inc = nanmax(inc, fabs(v - Uold[m * S + p]));
    un = nanmax(un, fabs(v));
  }
  block_max2(inc, un, red);
  if (threadIdx.x == 0) {
    atomicMax(&maxima[2 * m], (unsigned long long)__double_as_longlong(inc));
    atomicMax(&maxima[2 * m + 1], (unsigned long long)__double_as_longlong(un));
  }
}

int pow2_at_least(int n) {
  int p = 64;
  while (p < n) p <<= 1;
  return p;
}

unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384)); }

double from_bits(unsigned long long b) {
  double d;
  std::memcpy(&d, &b, sizeof d);
  return d;
}

}  // namespace

struct NLState {
  klecgc_model mp;
  int64_t M = 0;
  int n = 0, K = 0, P = 0;
  double dT = 0, dt = 0, ntol = 0;
  int nmax = 0;
  const double* coef = nullptr;
  unsigned int* fail = nullptr;      // [M]
  unsigned long long* counts = nullptr;  // [3]: Newton steps, backward-Euler steps, steps that hit the cap
  double* G = nullptr;               // [M][N][n]
  double* Uold = nullptr;            // [M][N][n]
  double* D = nullptr;               // [M][N][n]
  double* jbar = nullptr;            // [M][3][n]
  cplx* spec = nullptr;              // [M][K][n]
  unsigned long long* nmx = nullptr; // [2M]
  SliceTables tb{};
  std::vector<int64_t> newton_its;   // per sample, last correction
  int64_t newton_total = 0;
  int newton_max_seen = 0;
};

NLState* nl_prepare(klecgc_ctx* ctx, const klecgc_model& mp, const double* c, int64_t M, bool need_cgc) {
  auto* s = new NLState;
  try {
    s->mp = mp;
    s->M = M;
    s->n = mp.n;
    s->K = model_bins(mp.N);
    s->P = pow2_at_least(mp.n);
    s->dT = mp.T / mp.N;
    s->dt = s->dT / mp.J;
    s->ntol = mp.newton_tol > 0.0 ? mp.newton_tol : 1e-13;
    s->nmax = mp.newton_max_iter > 0 ? mp.newton_max_iter : 50;
    s->coef = c;
    s->newton_its.assign((size_t)M, 0);
    const size_t st_b = sizeof(double) * (size_t)M * mp.N * mp.n;
    const size_t small_b = sizeof(unsigned int) * (size_t)M + sizeof(double) * 3 * (size_t)mp.N +
                           sizeof(unsigned long long) * 2 * (size_t)M + 2048;
    char* sm = (char*)ctx->ws.get(WS_MODEL_SMALL, small_b);
    s->fail = (unsigned int*)sm;
    sm += (sizeof(unsigned int) * (size_t)M + 255) / 256 * 256;
    double* slt = (double*)sm;
    sm += (sizeof(double) * 3 * (size_t)mp.N + 255) / 256 * 256;
    s->nmx = (unsigned long long*)sm;
    sm += (sizeof(unsigned long long) * 2 * (size_t)M + 255) / 256 * 256;
    s->counts = (unsigned long long*)sm;
    KC_TRY_HIP(hipMemsetAsync(s->fail, 0, sizeof(unsigned int) * (size_t)M, ctx->stream));
    KC_TRY_HIP(hipMemsetAsync(s->counts, 0, sizeof(unsigned long long) * 3, ctx->stream));
    if (need_cgc) {
      s->tb = slice_tables(ctx, mp.N, mp.alpha, slt);
      char* big = (char*)ctx->ws.get(WS_MODEL_STATE, 3 * st_b + sizeof(double) * 3 * (size_t)M * mp.n);
      s->G = (double*)big;
      s->Uold = (double*)(big + st_b);
      s->D = (double*)(big + 2 * st_b);
      s->jbar = (double*)(big + 3 * st_b);
      s->spec = (cplx*)ctx->ws.get(WS_MODEL_SPEC, sizeof(cplx) * (size_t)M * s->K * mp.n);
    }
  } catch (...) {
    delete s;
    throw;
  }
  return s;
}

void nl_release(NLState* s) { delete s; }

void nl_initial_value(klecgc_ctx* ctx, const klecgc_model& mp, int64_t M, double* u0) {
  nl_u0_kernel<<<grid_of(M * mp.n), 256, 0, ctx->stream>>>(mp.model, mp.n, M, u0);
  KC_LAUNCH_CHECK();
}

// sweep: mode 0 direct, 1 shift, 2 twisted (see nl_sweep_kernel)
void nl_sweep(klecgc_ctx* ctx, NLState* s, const int32_t* list, int64_t nlist, const double* base, const double* u0,
              int mode, int s_lo, int nsl, bool coarse, double* out) {
  if (nlist <= 0 || nsl <= 0) return;
  const int P = s->P;
  KC_REQUIRE(P <= 1024, KC_EUNSUPPORTED, "the nonlinear models take n <= 1024");
  const size_t lds = sizeof(double) * (9 * (size_t)P + 32);
  timed(ctx, KT_FINE, [&] {
    nl_sweep_kernel<<<(unsigned)(nlist * nsl), P, lds, ctx->stream>>>(
        s->mp.model, s->n, s->coef, list, base, u0, mode, s->mp.alpha, s_lo, nsl, s->mp.N, coarse ? 1 : s->mp.J,
        coarse ? s->dT : s->dt, s->ntol, s->nmax, out, s->fail, s->counts);
  });
  KC_LAUNCH_CHECK();
}

// Coarse grid correction for the listed samples: U <- the Newton-CGC iterate from U^k = U and
// the fine results Fv; maxima[2m], [2m+1] = max |U^{k+1} - U^k|, max |U^{k+1}|.  `hlist` is the
// same list on the host.
void nl_correct(klecgc_ctx* ctx, NLState* s, const int32_t* list, const std::vector<int32_t>& hlist,
                int32_t* dev_newton_list, const double* Fv, double* U, unsigned long long* maxima) {
  const int64_t nl = (int64_t)hlist.size();
  if (nl == 0) return;
  hipStream_t st = ctx->stream;
  const int N = s->mp.N, n = s->n, K = s->K;
  const int64_t S = (int64_t)N * n;
  // G(z_s) on every slice, z_0 = alpha U_{N-1}, z_s = U_{s-1}; b = Fv - G
  nl_sweep(ctx, s, list, nl, U, nullptr, 2, 0, N, true, s->G);
  nl_copy_kernel<<<grid_of(nl * S), 256, 0, st>>>(list, nl, S, U, s->Uold);
  KC_LAUNCH_CHECK();
  std::vector<int32_t> cur = hlist, keep;
  std::vector<unsigned long long> mx;
  const double aroot = std::pow(s->mp.alpha, 1.0 / N);
  for (int l = 1; l <= s->nmax && !cur.empty(); ++l) {
    const int64_t nc = (int64_t)cur.size();
    KC_TRY_HIP(hipMemcpyAsync(dev_newton_list, cur.data(), sizeof(int32_t) * nc, hipMemcpyHostToDevice, st));
    KC_TRY_HIP(hipMemsetAsync(s->nmx, 0, sizeof(unsigned long long) * 2 * s->M, st));
    timed(ctx, KT_DEFECT, [&] {
      nl_avgjac_kernel<<<dim3((unsigned)((n + 255) / 256), (unsigned)nc), 256, 0, st>>>(
          s->mp.model, n, s->coef, dev_newton_list, N, U, Fv, s->G, s->jbar);
      nl_newton_rhs_kernel<<<dim3((unsigned)((n + 255) / 256), (unsigned)N, (unsigned)nc), 256, 0, st>>>(
          s->mp.model, n, s->coef, dev_newton_list, N, s->mp.alpha, s->dT, U, Fv, s->G, s->D);
    });
    KC_LAUNCH_CHECK();
    timed(ctx, KT_FFT_FWD, [&] { launch_slice_dft(st, s->D, dev_newton_list, nc, N, n, s->tb, s->spec); });
    timed(ctx, KT_SHIFTED, [&] {
      nl_shift_solve_kernel<<<(unsigned)(nc * K), s->P, sizeof(cplx) * 8 * (size_t)s->P, st>>>(
          n, dev_newton_list, K, N, aroot, s->dT, s->jbar, s->spec);
    });
    KC_LAUNCH_CHECK();
    timed(ctx, KT_FFT_INV, [&] { launch_slice_idft(st, s->spec, dev_newton_list, nc, N, n, s->tb, U, true, s->nmx); });
    mx.resize(2 * (size_t)s->M);
    KC_TRY_HIP(hipMemcpyAsync(mx.data(), s->nmx, sizeof(unsigned long long) * mx.size(), hipMemcpyDeviceToHost, st));
    KC_TRY_HIP(hipStreamSynchronize(st));
    keep.clear();
    for (int32_t m : cur) {
      const double d = from_bits(mx[2 * (size_t)m]), u = from_bits(mx[2 * (size_t)m + 1]);
      s->newton_its[m] = l;
      const bool done = d <= s->ntol * std::fmax(u, 1.0) || !std::isfinite(d);
      if (!done) keep.push_back(m);
    }
    s->newton_total += nc;
    s->newton_max_seen = std::max(s->newton_max_seen, l);
    cur.swap(keep);
  }
  if (maxima) {
    nl_increment_kernel<<<dim3((unsigned)std::min<int64_t>((S + 255) / 256, 64), (unsigned)nl), 256, 0, st>>>(
        list, S, U, s->Uold, maxima);
    KC_LAUNCH_CHECK();
  }
}

int nl_failed_samples(klecgc_ctx* ctx, NLState* s, std::vector<uint8_t>& bad) {
  std::vector<unsigned int> h((size_t)s->M);
  KC_TRY_HIP(hipMemcpyAsync(h.data(), s->fail, sizeof(unsigned int) * h.size(), hipMemcpyDeviceToHost, ctx->stream));
  KC_TRY_HIP(hipStreamSynchronize(ctx->stream));
  bad.assign((size_t)s->M, 0);
  int any = 0;
  for (int64_t m = 0; m < s->M; ++m) {
    bad[m] = h[m] != 0;
    any |= bad[m];
  }
  return any;
}

const std::vector<int64_t>& nl_newton_counts(const NLState* s) { return s->newton_its; }
void nl_sweep_counts(klecgc_ctx* ctx, const NLState* s, int64_t* newton, int64_t* steps, int64_t* capped) {
  unsigned long long h[3] = {0, 0, 0};
  KC_TRY_HIP(hipMemcpyAsync(h, s->counts, sizeof h, hipMemcpyDeviceToHost, ctx->stream));
  KC_TRY_HIP(hipStreamSynchronize(ctx->stream));
  *newton = (int64_t)h[0];
  *steps = (int64_t)h[1];
  *capped = (int64_t)h[2];
}
int64_t nl_newton_total(const NLState* s) { return s->newton_total; }
int nl_newton_max(const NLState* s) { return s->newton_max_seen; }

}  // namespace kc
