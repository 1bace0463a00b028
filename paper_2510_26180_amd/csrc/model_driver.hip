// Drivers of the Section 5 model problems: the building blocks (F over all slices, the
// sequential G and F sweeps, one coarse grid correction) and the parareal loops of
// Algorithms 1-3 for a batch of samples, each sample with its own parameter.
//
// The loop keeps a host-side list of the samples still iterating; every kernel of an
// iteration works on the listed samples only, and the host reads the per-sample increment
// maxima once per iteration to update the list (these problems are small: the per-iteration
// read-back costs microseconds next to the fine sweep).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "models.h"
#include "reduce.h"

namespace kc {

namespace {

// Algorithm 1 correction on slice s: Unew[m][s] = Gn[m][s] + F[m][s] - Go[m][s]
__global__ void seq_combine_kernel(const int32_t* __restrict__ list, int64_t nlist, int N, int64_t Nx, int s,
                                   const double* __restrict__ Gn, const double* __restrict__ Fv,
                                   const double* __restrict__ Go, double* __restrict__ Unew) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nlist * Nx; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = list[t / Nx];
    const int64_t o = (m * N + s) * Nx + t % Nx;
    Unew[o] = Gn[o] + Fv[o] - Go[o];
  }
}

// U <- Unew for the listed samples, with maxima[2m] = max |Unew - U|, maxima[2m+1] = max |Unew|
__global__ __launch_bounds__(256) void commit_kernel(const int32_t* __restrict__ list, int N, int64_t Nx,
                                                     const double* __restrict__ Unew, double* __restrict__ U,
                                                     unsigned long long* __restrict__ maxima) {
  __shared__ double red[8];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  const int64_t m = list[blockIdx.z];
  double inc = 0.0, un = 0.0;
  if (p < Nx) {
    const int64_t o = (m * N + s) * Nx + p;
    const double v = Unew[o];
    inc = fabs(v - U[o]);
    un = fabs(v);
    U[o] = v;
  }
  double v[2] = {inc, un};
  const bool mx[2] = {true, true};
  block_reduce<2>(v, mx, red);
  if (threadIdx.x == 0) {
    atomicMax(&maxima[2 * m], (unsigned long long)__double_as_longlong(v[0]));
    atomicMax(&maxima[2 * m + 1], (unsigned long long)__double_as_longlong(v[1]));
  }
}

unsigned grid1(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384)); }

double bits_to_double(unsigned long long b) {
  double d;
  std::memcpy(&d, &b, sizeof d);
  return d;
}

// The operations the drivers need from a model: F or G on a range of slices, one coarse
// grid correction of the listed samples, the model's initial value, and the samples a
// solver flagged (unusable pivots, Newton iterations that hit their cap).
struct Ops {
  virtual ~Ops() = default;
  virtual void sweep(const int32_t* list, int64_t nlist, const double* base, const double* u0, bool shift,
                     int s_lo, int nsl, bool coarse, double* out) = 0;
  virtual void correct(const int32_t* list, const std::vector<int32_t>& hlist, const double* Fv, double* U,
                       unsigned long long* maxima) = 0;
  virtual void initial_value(int64_t M, double* u0) = 0;
  virtual int flagged(std::vector<uint8_t>& bad) = 0;
  virtual int64_t newton_its(int64_t m) const { return 1; }
  virtual int flagged_code() const { return KC_ENONFINITE; }
  // counters for klecgc_last_stats (nonlinear models): [0] Newton steps of the backward-Euler
  // steps of all sweeps, [2] those backward-Euler steps (both summed over systems), [4] Newton
  // steps of the corrections summed over samples, [7] the most one correction of one sample
  // took, [10] backward-Euler steps whose Newton iteration reached its cap
  virtual void report(int64_t* stats) {}
};

struct AdeOps : Ops {
  klecgc_ctx* ctx;
  klecgc_model mp;
  AdeState* s;
  AdeOps(klecgc_ctx* c, const klecgc_model& m, const double* coef, int64_t M, bool coarse, bool cgc)
      : ctx(c), mp(m), s(ade_prepare(c, m, coef, M, coarse, cgc)) {}
  ~AdeOps() override { ade_release(s); }
  void sweep(const int32_t* list, int64_t nlist, const double* base, const double* u0, bool shift, int s_lo, int nsl,
             bool coarse, double* out) override {
    ade_sweep(ctx, s, list, nlist, AdeSweep{base, u0, shift, s_lo, nsl, coarse, out});
  }
  void correct(const int32_t* list, const std::vector<int32_t>& hlist, const double* Fv, double* U,
               unsigned long long* maxima) override {
    ade_correct(ctx, s, list, (int64_t)hlist.size(), Fv, U, maxima);
  }
  void initial_value(int64_t M, double* u0) override { ade_initial_value(ctx, mp, M, u0); }
  int flagged(std::vector<uint8_t>& bad) override { return ade_bad_samples(ctx, s, bad); }
};

struct NLOps : Ops {
  klecgc_ctx* ctx;
  klecgc_model mp;
  NLState* s;
  int32_t* newton_list;
  int64_t s_M;
  NLOps(klecgc_ctx* c, const klecgc_model& m, const double* coef, int64_t M, bool cgc, int32_t* scratch_list)
      : ctx(c), mp(m), s(nl_prepare(c, m, coef, M, cgc)), newton_list(scratch_list), s_M(M) {}
  ~NLOps() override { nl_release(s); }
  void sweep(const int32_t* list, int64_t nlist, const double* base, const double* u0, bool shift, int s_lo, int nsl,
             bool coarse, double* out) override {
    nl_sweep(ctx, s, list, nlist, base, u0, shift ? 1 : 0, s_lo, nsl, coarse, out);
  }
  void correct(const int32_t* list, const std::vector<int32_t>& hlist, const double* Fv, double* U,
               unsigned long long* maxima) override {
    nl_correct(ctx, s, list, hlist, newton_list, Fv, U, maxima);
  }
  void initial_value(int64_t M, double* u0) override { nl_initial_value(ctx, mp, M, u0); }
  // a backward-Euler Newton iteration at its cap keeps its last iterate: counted, not an error
  int flagged(std::vector<uint8_t>& bad) override {
    bad.assign((size_t)s_M, 0);
    return 0;
  }
  int64_t newton_its(int64_t m) const override { return nl_newton_counts(s)[m]; }
  void report(int64_t* stats) override {
    stats[4] = nl_newton_total(s);
    stats[7] = nl_newton_max(s);
    nl_sweep_counts(ctx, s, &stats[0], &stats[2], &stats[10]);
  }
};

// device scratch of the drivers: u0 [M][Nx], two lists [M], maxima [2M], err [M][N], states
struct DriverBufs {
  double* u0 = nullptr;
  int32_t* list = nullptr;
  int32_t* list2 = nullptr;
  unsigned long long* maxima = nullptr;
  unsigned long long* err = nullptr;
  double* A = nullptr;
  double* B = nullptr;
  double* C = nullptr;
};

DriverBufs driver_bufs(klecgc_ctx* ctx, int64_t M, int N, int64_t Nx, int n_states) {
  const size_t u0_b = sizeof(double) * (size_t)M * Nx;
  const size_t list_b = (sizeof(int32_t) * (size_t)M + 255) / 256 * 256;
  const size_t mx_b = sizeof(unsigned long long) * 2 * (size_t)M;
  const size_t err_b = (sizeof(unsigned long long) * (size_t)M * N + 255) / 256 * 256;
  const size_t st_b = sizeof(double) * (size_t)M * N * Nx;
  char* p = (char*)ctx->ws.get(WS_MODEL_AUX, u0_b + 2 * list_b + mx_b + err_b + st_b * n_states + 1024);
  DriverBufs b;
  b.u0 = (double*)p;
  p += (u0_b + 255) / 256 * 256;
  b.list = (int32_t*)p;
  p += list_b;
  b.list2 = (int32_t*)p;
  p += list_b;
  b.maxima = (unsigned long long*)p;
  p += (mx_b + 255) / 256 * 256;
  b.err = (unsigned long long*)p;
  p += err_b;
  if (n_states > 0) b.A = (double*)p;
  if (n_states > 1) b.B = (double*)(p + st_b);
  if (n_states > 2) b.C = (double*)(p + 2 * st_b);
  return b;
}

std::unique_ptr<Ops> make_ops(klecgc_ctx* ctx, const klecgc_model& mp, const double* c, int64_t M, bool coarse,
                              bool cgc, const DriverBufs& b) {
  if (mp.model == KC_MODEL_ADE_P1) return std::unique_ptr<Ops>(new AdeOps(ctx, mp, c, M, coarse, cgc));
  return std::unique_ptr<Ops>(new NLOps(ctx, mp, c, M, cgc, b.list2));
}

}  // namespace

void validate_model(const klecgc_model& mp) {
  KC_REQUIRE(mp.model == KC_MODEL_ADE_P1 || mp.model == KC_MODEL_BURGERS || mp.model == KC_MODEL_ALLEN_CAHN,
             KC_EINVAL, "unknown model");
  KC_REQUIRE(mp.T > 0.0 && std::isfinite(mp.T), KC_EINVAL, "T must be > 0");
  KC_REQUIRE(mp.N >= 2 && mp.N <= 64, KC_EINVAL, "N must lie in [2, 64]");
  KC_REQUIRE(mp.J >= 1, KC_EINVAL, "J must be >= 1");
  KC_REQUIRE(mp.alpha > 0.0 && mp.alpha < 1.0, KC_EINVAL, "alpha must lie in (0, 1)");
  KC_REQUIRE(mp.tol >= 0.0 && std::isfinite(mp.tol), KC_EINVAL, "tol must be >= 0");
  KC_REQUIRE(mp.max_iter >= 1 && mp.max_iter <= 1000, KC_EINVAL, "max_iter must lie in [1, 1000]");
  KC_REQUIRE(mp.newton_tol >= 0.0 && mp.newton_max_iter >= 0, KC_EINVAL, "bad Newton controls");
  if (mp.model == KC_MODEL_ADE_P1) {
    KC_REQUIRE(mp.n >= 2, KC_EINVAL, "n must be >= 2");
    KC_REQUIRE(mp.n <= 31, KC_EUNSUPPORTED, "the banded finite-element solver takes n <= 31");
    KC_REQUIRE(std::isfinite(mp.beta), KC_EINVAL, "beta must be finite");
  } else {
    KC_REQUIRE(mp.n >= 2, KC_EINVAL, "n must be >= 2");
    KC_REQUIRE(mp.n <= 512, KC_EUNSUPPORTED, "the nonlinear models take n <= 512");
  }
}

int model_fine_impl(klecgc_ctx* ctx, const klecgc_model& mp, const double* c, const double* start, int64_t M,
                    double* end) {
  DriverBufs b = driver_bufs(ctx, M, mp.N, model_nx(mp), 0);
  auto ops = make_ops(ctx, mp, c, M, false, false, b);
  ops->sweep(nullptr, M, start, nullptr, false, 0, mp.N, false, end);
  ops->report(ctx->stats);
  std::vector<uint8_t> bad;
  return ops->flagged(bad) ? ops->flagged_code() : KC_OK;
}

static int sequential_sweep(klecgc_ctx* ctx, const klecgc_model& mp, const double* c, const double* u0, int64_t M,
                            double* U, bool coarse) {
  DriverBufs b = driver_bufs(ctx, M, mp.N, model_nx(mp), 0);
  auto ops = make_ops(ctx, mp, c, M, coarse, false, b);
  if (!u0) {
    ops->initial_value(M, b.u0);
    u0 = b.u0;
  }
  for (int s = 0; s < mp.N; ++s) ops->sweep(nullptr, M, U, u0, true, s, 1, coarse, U);
  ops->report(ctx->stats);
  std::vector<uint8_t> bad;
  return ops->flagged(bad) ? ops->flagged_code() : KC_OK;
}

int model_coarse_impl(klecgc_ctx* ctx, const klecgc_model& mp, const double* c, const double* u0, int64_t M,
                      double* U) {
  return sequential_sweep(ctx, mp, c, u0, M, U, true);
}

int model_serial_fine_impl(klecgc_ctx* ctx, const klecgc_model& mp, const double* c, const double* u0, int64_t M,
                           double* U) {
  return sequential_sweep(ctx, mp, c, u0, M, U, false);
}

int model_cgc_impl(klecgc_ctx* ctx, const klecgc_model& mp, const double* c, const double* Uk, const double* Fv,
                   int64_t M, double* Unew, int32_t* newton_its) {
  const int64_t Nx = model_nx(mp);
  DriverBufs b = driver_bufs(ctx, M, mp.N, Nx, 0);
  auto ops = make_ops(ctx, mp, c, M, false, true, b);
  if (Unew != Uk)
    KC_TRY_HIP(hipMemcpyAsync(Unew, Uk, sizeof(double) * (size_t)M * mp.N * Nx, hipMemcpyDeviceToDevice, ctx->stream));
  std::vector<int32_t> all((size_t)M);
  for (int64_t m = 0; m < M; ++m) all[m] = (int32_t)m;
  KC_TRY_HIP(hipMemcpyAsync(b.list, all.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice, ctx->stream));
  ops->correct(b.list, all, Fv, Unew, nullptr);
  KC_TRY_HIP(hipStreamSynchronize(ctx->stream));
  if (newton_its)
    for (int64_t m = 0; m < M; ++m) newton_its[m] = (int32_t)ops->newton_its(m);
  ops->report(ctx->stats);
  std::vector<uint8_t> bad;
  return ops->flagged(bad) ? ops->flagged_code() : KC_OK;
}

int model_parareal_impl(klecgc_ctx* ctx, const klecgc_model& mp, const ModelSolveArgs& a) {
  hipStream_t st = ctx->stream;
  const int64_t M = a.M;
  const int N = mp.N;
  const int64_t Nx = model_nx(mp);
  const int64_t S = (int64_t)N * Nx;
  const GuessArgs& g = a.guess;
  const bool seq = a.sequential;
  // states: Fbuf; Algorithm 1 also Gold and Unew
  DriverBufs b = driver_bufs(ctx, M, N, Nx, seq ? 3 : 1);
  auto ops = make_ops(ctx, mp, a.c, M, seq || g.init == KC_INIT_COARSE, !seq, b);
  double* Fbuf = b.A;
  const double* u0 = a.u0;
  if (!u0) {
    ops->initial_value(M, b.u0);
    u0 = b.u0;
  }
  double* U = a.U;
  switch (g.init) {
    case KC_INIT_GIVEN:
      KC_TRY_HIP(hipMemcpyAsync(U, g.given, sizeof(double) * M * S, hipMemcpyDeviceToDevice, st));
      break;
    case KC_INIT_ZERO:
      KC_TRY_HIP(hipMemsetAsync(U, 0, sizeof(double) * M * S, st));
      break;
    case KC_INIT_RANDOM:
      launch_random_guess(st, g.seed, M * S, U);
      break;
    case KC_INIT_COARSE:
      for (int s = 0; s < N; ++s) ops->sweep(nullptr, M, U, u0, true, s, 1, true, U);
      break;
    case KC_INIT_GPC:
      KC_REQUIRE(g.gpc && g.xi, KC_EINVAL, "KC_INIT_GPC needs a gPC surrogate and xi");
      KC_REQUIRE(g.gpc->L == S, KC_EINVAL, "the gPC surrogate's state length differs from N * Nx");
      gpc_predict_impl(ctx, g.gpc, g.xi, M, U);
      break;
    default:
      throw Error{KC_EUNSUPPORTED, "initial guess mode not available for the model problems"};
  }
  std::vector<uint8_t> bad;
  ops->flagged(bad);
  std::vector<int32_t> list;
  for (int64_t m = 0; m < M; ++m) {
    a.iters[m] = 0;
    a.status[m] = bad[m] ? KC_SAMPLE_NONFINITE : KC_SAMPLE_MAXITER;
    if (!bad[m]) list.push_back((int32_t)m);
  }
  if (a.delta_hist) std::fill(a.delta_hist, a.delta_hist + M * mp.max_iter, 0.0);
  if (a.err_hist) std::fill(a.err_hist, a.err_hist + M * (mp.max_iter + 1) * N, 0.0);
  std::vector<unsigned long long> errh;
  auto record_errors = [&](int k, const int32_t* dlist, int64_t nl) {
    if (!a.err_hist || !a.ref) return;
    KC_TRY_HIP(hipMemsetAsync(b.err, 0, sizeof(unsigned long long) * M * N, st));
    launch_slice_error(st, U, a.ref, dlist, nl, N, Nx, b.err);
    errh.resize((size_t)M * N);
    KC_TRY_HIP(hipMemcpyAsync(errh.data(), b.err, sizeof(unsigned long long) * errh.size(), hipMemcpyDeviceToHost, st));
    KC_TRY_HIP(hipStreamSynchronize(st));
    for (int64_t i = 0; i < nl; ++i) {
      const int64_t m = list[i];
      for (int s = 0; s < N; ++s)
        a.err_hist[((size_t)m * (mp.max_iter + 1) + k) * N + s] = bits_to_double(errh[(size_t)m * N + s]);
    }
  };
  // the first slice's fine result F(u0) does not change between iterations
  if (!list.empty()) {
    KC_TRY_HIP(hipMemcpyAsync(b.list, list.data(), sizeof(int32_t) * list.size(), hipMemcpyHostToDevice, st));
    record_errors(0, b.list, (int64_t)list.size());
    ops->sweep(b.list, (int64_t)list.size(), U, u0, true, 0, 1, false, Fbuf);
  }
  std::vector<unsigned long long> mx;
  for (int it = 0; it < mp.max_iter && !list.empty(); ++it) {
    const int64_t nl = (int64_t)list.size();
    KC_TRY_HIP(hipMemcpyAsync(b.list, list.data(), sizeof(int32_t) * nl, hipMemcpyHostToDevice, st));
    KC_TRY_HIP(hipMemsetAsync(b.maxima, 0, sizeof(unsigned long long) * 2 * M, st));
    // step 1: fine propagation of slices 1..N-1 from the current iterate
    ops->sweep(b.list, nl, U, u0, true, 1, N - 1, false, Fbuf);
    if (!seq) {
      // step 2 (Algorithms 2/3): the diagonalised CGC (one linear solve, or the Newton iteration)
      ops->correct(b.list, list, Fbuf, U, b.maxima);
    } else {
      // step 2 (Algorithm 1): Gold = G(U^k_{s-1}) on all slices, then the sequential sweep
      double* Gold = b.B;
      double* Unew = b.C;
      ops->sweep(b.list, nl, U, u0, true, 0, N, true, Gold);
      for (int s = 0; s < N; ++s) {
        ops->sweep(b.list, nl, Unew, u0, true, s, 1, true, Unew);
        seq_combine_kernel<<<grid1(nl * Nx), 256, 0, st>>>(b.list, nl, N, Nx, s, Unew, Fbuf, Gold, Unew);
        KC_LAUNCH_CHECK();
      }
      dim3 gc((unsigned)((Nx + 255) / 256), (unsigned)N, (unsigned)nl);
      commit_kernel<<<gc, 256, 0, st>>>(b.list, N, Nx, Unew, U, b.maxima);
      KC_LAUNCH_CHECK();
    }
    record_errors(it + 1, b.list, nl);
    mx.resize(2 * (size_t)M);
    KC_TRY_HIP(hipMemcpyAsync(mx.data(), b.maxima, sizeof(unsigned long long) * mx.size(), hipMemcpyDeviceToHost, st));
    KC_TRY_HIP(hipStreamSynchronize(st));
    std::vector<int32_t> keep;
    for (int64_t i = 0; i < nl; ++i) {
      const int64_t m = list[i];
      const double inc = bits_to_double(mx[2 * m]), un = bits_to_double(mx[2 * m + 1]);
      const double delta = inc / (un > 0.0 ? un : 1.0);
      a.iters[m] = it + 1;
      if (a.delta_hist) a.delta_hist[m * mp.max_iter + it] = delta;
      if (!std::isfinite(delta)) {
        a.status[m] = KC_SAMPLE_NONFINITE;
      } else if (mp.tol > 0.0 && delta <= mp.tol) {
        a.status[m] = KC_SAMPLE_CONVERGED;
      } else {
        keep.push_back((int32_t)m);
      }
    }
    list.swap(keep);
  }
  ops->report(ctx->stats);
  // rows of the error history after a sample's stop repeat its last iterate's errors
  if (a.err_hist && a.ref)
    for (int64_t m = 0; m < M; ++m)
      for (int k = a.iters[m] + 1; k <= mp.max_iter; ++k)
        for (int s = 0; s < N; ++s)
          a.err_hist[((size_t)m * (mp.max_iter + 1) + k) * N + s] =
              a.err_hist[((size_t)m * (mp.max_iter + 1) + a.iters[m]) * N + s];
  return KC_OK;
}

}  // namespace kc
