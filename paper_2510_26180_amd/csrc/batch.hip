// Parareal driver (Algorithm 2 iterated as in Algorithm 3 step 7) for one or several
// uniform classes of samples, with the convergence test on the device.
//
// Each iteration of a class enqueues: fine sweep over its active (sample, slice) pairs,
// defect, forward slice FFT, shifted solves, inverse FFT accumulating the correction
// into U together with per-sample maxima, and `converge_kernel`, which turns the maxima
// into the increment delta = max|U^{k+1}-U^k| / max|U^{k+1}|, records it, and retires the
// sample (converged, non-finite or at the iteration cap) by clearing its mask.  No
// iteration needs the host, so after one eager iteration (which also sizes every
// workspace) the iteration of all classes is captured once into a hipGraph, one branch
// per class on its own stream, and replayed until every sample has retired.
//
// Ragged batches (samples of different grid size n and slice count N) are grouped into
// classes of equal (n, N); each class is gathered into contiguous buffers, run on its own
// context and stream, and scattered back.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <functional>
#include <map>
#include <mutex>
#include <memory>
#include <numeric>
#include <thread>
#include <vector>

#include "common.h"
#include "models.h"
#include "reduce.h"

namespace kc {

namespace {

__global__ void converge_kernel(int64_t M, int max_iter, double tol, unsigned long long* __restrict__ maxima,
                                uint8_t* __restrict__ active, int32_t* __restrict__ its,
                                int32_t* __restrict__ status, double* __restrict__ hist,
                                unsigned long long* __restrict__ tconv, int* __restrict__ counts, int cls) {
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < M; m += (int64_t)gridDim.x * blockDim.x) {
    if (!active[m]) continue;
    const double cmax = __longlong_as_double((long long)maxima[2 * m]);
    const double umax = __longlong_as_double((long long)maxima[2 * m + 1]);
    maxima[2 * m] = 0ull;
    maxima[2 * m + 1] = 0ull;
    const double delta = cmax / (umax > 0 ? umax : 1.0);
    const int k = its[m];
    its[m] = k + 1;
    if (hist) hist[m * max_iter + k] = delta;
    bool stop = false;
    if (!isfinite(delta)) {
      status[m] = KC_SAMPLE_NONFINITE;
      stop = true;
    } else if (delta <= tol) {
      status[m] = KC_SAMPLE_CONVERGED;
      stop = true;
    } else if (k + 1 >= max_iter) {
      stop = true;  // status stays KC_SAMPLE_MAXITER
    }
    if (stop) {
      active[m] = 0;
      if (tconv) tconv[m] = wall_clock64();
      atomicSub(&counts[cls], 1);
      atomicSub(&counts[0], 1);
    }
  }
}

// per-class state set-up: active = 1, its = 0, status = MAXITER, maxima = 0
__global__ void class_init_kernel(int64_t M, uint8_t* active, int32_t* its, int32_t* status,
                                  unsigned long long* maxima) {
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < M; m += (int64_t)gridDim.x * blockDim.x) {
    active[m] = 1;
    its[m] = 0;
    status[m] = KC_SAMPLE_MAXITER;
    maxima[2 * m] = 0ull;
    maxima[2 * m + 1] = 0ull;
  }
}

__global__ void stamp_kernel(unsigned long long* t) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *t = wall_clock64();
}

// dst[j][0..len) = src[off[j] .. off[j]+len), j < R   (and the reverse for scatter)
__global__ void gather_rows_kernel(const double* __restrict__ src, const int64_t* __restrict__ off, int64_t len,
                                   int64_t R, double* __restrict__ dst) {
  const int64_t j = blockIdx.y;
  if (j >= R) return;
  const double* s = src + off[j];
  double* d = dst + j * len;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

__global__ void scatter_rows_kernel(const double* __restrict__ src, const int64_t* __restrict__ off, int64_t len,
                                    int64_t R, double* __restrict__ dst) {
  const int64_t j = blockIdx.y;
  if (j >= R) return;
  const double* s = src + j * len;
  double* d = dst + off[j];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

// The random initial guess: entry i is the SplitMix64 output (Steele, Lea and Flood, OOPSLA
// 2014) of the state seed + (i + 1) * golden (mod 2^64), its top 53 bits scaled by 2^-53.
__global__ void random_guess_kernel(unsigned long long seed, int64_t n, double* __restrict__ U) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    unsigned long long z = seed + (unsigned long long)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    U[i] = (double)(z >> 11) * 0x1.0p-53;
  }
}

// Continuity defects of two guesses after a fine sweep on each: for sample m,
// mx[4m + 0] = max |F_l - U_l|, mx[4m + 1] = max |U_l|, mx[4m + 2], mx[4m + 3] the same for the
// second guess (F_g - U_g, U_g), as ordered bit patterns of non-negative doubles (NaN wins).
__global__ __launch_bounds__(256) void guess_defect_kernel(const double* __restrict__ Fl, const double* __restrict__ Ul,
                                                           const double* __restrict__ Fg, const double* __restrict__ Ug,
                                                           int64_t S, unsigned long long* __restrict__ mx) {
  const int64_t m = blockIdx.y;
  const int64_t o = m * S;
  double jl = 0.0, ul = 0.0, jg = 0.0, ug = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S; i += (int64_t)gridDim.x * blockDim.x) {
    const double u = Ul[o + i], v = Ug[o + i];
    jl = nanmax(jl, fabs(Fl[o + i] - u));
    ul = nanmax(ul, fabs(u));
    jg = nanmax(jg, fabs(Fg[o + i] - v));
    ug = nanmax(ug, fabs(v));
  }
  jl = wave_nanmax(jl);
  ul = wave_nanmax(ul);
  jg = wave_nanmax(jg);
  ug = wave_nanmax(ug);
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&mx[4 * m + 0], (unsigned long long)__double_as_longlong(jl));
    atomicMax(&mx[4 * m + 1], (unsigned long long)__double_as_longlong(ul));
    atomicMax(&mx[4 * m + 2], (unsigned long long)__double_as_longlong(jg));
    atomicMax(&mx[4 * m + 3], (unsigned long long)__double_as_longlong(ug));
  }
}

// The fallback rule: keep the learned guess unless the fallback's defect is strictly
// smaller, or the learned one's is NaN and the fallback's is not.  A zero maximum of |U|
// divides by 1.  use[m] = 1 selects the fallback.
__global__ void guess_choose_kernel(const unsigned long long* __restrict__ mx, int64_t M, int32_t* __restrict__ use) {
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < M; m += (int64_t)gridDim.x * blockDim.x) {
    const double jl = __longlong_as_double((long long)mx[4 * m + 0]);
    const double ul = __longlong_as_double((long long)mx[4 * m + 1]);
    const double jg = __longlong_as_double((long long)mx[4 * m + 2]);
    const double ug = __longlong_as_double((long long)mx[4 * m + 3]);
    const double dl = jl / (ul > 0 ? ul : 1.0);
    const double dg = jg / (ug > 0 ? ug : 1.0);
    use[m] = (dg < dl || (isnan(dl) && !isnan(dg))) ? 1 : 0;
  }
}

// U[m] = Ug[m] and F[m] = Fg[m] for the samples with use[m] != 0
__global__ void guess_take_kernel(const int32_t* __restrict__ use, const double* __restrict__ Ug,
                                  const double* __restrict__ Fg, int64_t S, double* __restrict__ U,
                                  double* __restrict__ F) {
  const int64_t m = blockIdx.y;
  if (!use[m]) return;
  const int64_t o = m * S;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S; i += (int64_t)gridDim.x * blockDim.x) {
    U[o + i] = Ug[o + i];
    F[o + i] = Fg[o + i];
  }
}

__global__ void zero_kernel(double* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.0;
}

unsigned blocks_of(int64_t n, int64_t cap = 4096) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, cap));
}

void launch_rows(bool gather, hipStream_t s, const double* src, const int64_t* off, int64_t len, int64_t R,
                 double* dst) {
  for (int64_t r0 = 0; r0 < R; r0 += 65535) {
    const int64_t Rc = std::min<int64_t>(65535, R - r0);
    const dim3 grid(blocks_of(len, 64), (unsigned)Rc);
    if (gather)
      gather_rows_kernel<<<grid, 256, 0, s>>>(src, off + r0, len, Rc, dst + r0 * len);
    else
      scatter_rows_kernel<<<grid, 256, 0, s>>>(src + r0 * len, off + r0, len, Rc, dst);
    KC_LAUNCH_CHECK();
  }
}

// device state of one class (owned allocation)
struct ClassState {
  uint8_t* active = nullptr;
  int32_t* its = nullptr;
  int32_t* status = nullptr;
  double* hist = nullptr;
  unsigned long long* maxima = nullptr;
  unsigned long long* tconv = nullptr;
  void* base = nullptr;
  void alloc(int64_t M, int max_iter, bool want_hist) {
    const size_t b_act = (M + 255) / 256 * 256, b_i32 = (4 * M + 255) / 256 * 256;
    const size_t b_hist = want_hist ? (8 * (size_t)M * max_iter + 255) / 256 * 256 : 0;
    const size_t b_u64 = (8 * M + 255) / 256 * 256;
    const size_t total = b_act + 2 * b_i32 + b_hist + 3 * b_u64;
    if (hipMalloc(&base, total) != hipSuccess) {
      (void)hipGetLastError();
      base = nullptr;
      throw Error{KC_ENOMEM, "parareal driver state allocation failed"};
    }
    char* p = (char*)base;
    active = (uint8_t*)p;
    p += b_act;
    its = (int32_t*)p;
    p += b_i32;
    status = (int32_t*)p;
    p += b_i32;
    hist = want_hist ? (double*)p : nullptr;
    p += b_hist;
    maxima = (unsigned long long*)p;
    p += 2 * b_u64;
    tconv = (unsigned long long*)p;
  }
  ~ClassState() {
    if (base) (void)hipFree(base);
  }
};

}  // namespace

// One uniform class of samples: problem p (n, N fixed), M samples, faces a [M][Fc],
// states U [M][N][Nx] (initial guess on entry, iterate on exit).
struct ParaClass {
  klecgc_ctx* c = nullptr;  // execution context (its stream and workspace)
  klecgc_problem p{};
  klecgc_problem pb{};      // p with the default correction tolerance of the shifted solves
  int64_t M = 0;
  const double* a = nullptr;
  const double* u0 = nullptr;
  double* U = nullptr;
  ClassState st;
  int index = 1;            // slot in the device counter array (0 = all classes)
  bool fine_ready = false;  // the F buffer already holds iteration 0's fine sweep
  bool fine_external = false;  // its fine sweep runs in the driver's persistent launch
};

static void enqueue_iteration(ParaClass& pc, int k, int* counts, int& rc) {
  klecgc_ctx* c = pc.c;
  hipStream_t s = c->stream;
  const klecgc_problem& p = pc.p;
  const int64_t Nx = n_unknowns(p);
  const int64_t S = (int64_t)p.N * Nx;
  const int K = p.N / 2 + 1;
  double* Fv = (double*)c->ws.get(WS_FINE, sizeof(double) * pc.M * S);
  double* D = (double*)c->ws.get(WS_DEFECT, sizeof(double) * pc.M * S);
  double* spec = (double*)c->ws.get(WS_SPEC, sizeof(double) * 2 * pc.M * K * Nx);
  if (!(k == 0 && pc.fine_ready) && !pc.fine_external) {
    FineArgs fa{pc.a, pc.U, pc.u0, true, k > 0 ? 1 : 0, pc.st.active, Fv, pc.M};
    const int r = fine_propagate_impl(c, p, fa);
    if (r != KC_OK) rc = r;
  }
  int r;
  timed(c, KT_DEFECT, [&] { launch_defect(s, p, pc.a, Fv, pc.U, pc.st.active, pc.M, D); });
  timed(c, KT_FFT_FWD, [&] { launch_fft_forward(s, p, D, pc.st.active, pc.M, spec); });
  r = shifted_solve_impl(c, pc.pb, pc.a, pc.st.active, pc.M, spec);
  if (r != KC_OK) rc = r;
  timed(c, KT_FFT_INV, [&] { launch_fft_inverse(s, p, spec, pc.st.active, pc.M, pc.U, true, pc.st.maxima); });
  converge_kernel<<<blocks_of(pc.M), 256, 0, s>>>(pc.M, p.max_iter, p.tol, pc.st.maxima, pc.st.active, pc.st.its,
                                                  pc.st.status, pc.st.hist, pc.st.tconv, counts, pc.index);
  KC_LAUNCH_CHECK();
}

// an iteration of the class is a fixed sequence of launches (no host decisions inside)
static bool iteration_capturable(const ParaClass& pc) {
  if (pc.fine_external) return true;
  if (pc.p.dim == 1 || pc.p.precision != KC_PREC_F32_REFINED) return true;
  return fine_variant_for(pc.p.n, tuning_for(pc.c, pc.p.n).fine_variant) != KC_FINE_MG;
}

struct DriverOut {
  std::vector<int32_t> its, status;   // per class, concatenated in class order
  std::vector<double> hist;
  std::vector<unsigned long long> tconv;
  unsigned long long t0 = 0;
  int iterations = 0;                 // driver iterations (graph replays + 1)
  double graph_ms = 0;                // capture + instantiate time
};

// Runs the parareal iteration over the classes.  `main` is the stream that orders the
// whole run (the caller's); with use_graph the classes' iterations after the first are
// replayed from one captured graph.
// With `persistent`, the fine sweeps of every class that qualifies (persistent_eligible) run
// as one persistent launch per iteration on the ordering stream, ahead of the classes'
// branches.
static int run_classes(klecgc_ctx* ctx, std::vector<ParaClass*>& cls, bool use_graph, bool want_hist,
                       DriverOut& out, bool progress = false, bool persistent = false) {
  const auto t_start = std::chrono::steady_clock::now();
  auto report = [&](int k, int active) {
    if (!progress && !progress_enabled()) return;
    const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    std::fprintf(stderr, "[klecgc] parareal iteration %d: %d samples active, %.1f s\n", k, active, s);
    std::fflush(stderr);
  };
  hipStream_t main = ctx->stream;
  const int C = (int)cls.size();
  int max_iter = 1;
  int64_t total = 0;
  for (auto* pc : cls) {
    max_iter = std::max(max_iter, pc->p.max_iter);
    total += pc->M;
  }
  // device counters: [0] active samples of all classes, [1 + i] of class i; stamp at [C+1]
  char* cbuf = (char*)ctx->ws.get(WS_SMALL, 256 + sizeof(int) * (C + 1));
  unsigned long long* t0dev = (unsigned long long*)cbuf;
  int* counts = (int*)(cbuf + 256);
  std::vector<int> hc(C + 1);
  hc[0] = (int)total;
  for (int i = 0; i < C; ++i) hc[i + 1] = (int)cls[i]->M;
  KC_TRY_HIP(hipMemcpyAsync(counts, hc.data(), sizeof(int) * (C + 1), hipMemcpyHostToDevice, main));
  stamp_kernel<<<1, 64, 0, main>>>(t0dev);
  KC_LAUNCH_CHECK();
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join(C, nullptr);
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      if (*e) (void)hipEventDestroy(*e);
    }
  };
  KC_TRY_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
  EvGuard fg{&fork};
  std::vector<std::unique_ptr<EvGuard>> jg;
  for (int i = 0; i < C; ++i) {
    KC_TRY_HIP(hipEventCreateWithFlags(&join[i], hipEventDisableTiming));
    jg.emplace_back(new EvGuard{&join[i]});
  }
  // `order` is the stream that sequences the iterations: the caller's stream while
  // iterating eagerly, a driver-owned stream for the graph (capture is not allowed on
  // the legacy null stream a caller may pass)
  hipStream_t order = main;
  auto fork_all = [&]() {
    KC_TRY_HIP(hipEventRecord(fork, order));
    for (auto* pc : cls)
      if (pc->c->stream != order) KC_TRY_HIP(hipStreamWaitEvent(pc->c->stream, fork, 0));
  };
  auto join_all = [&]() {
    for (int i = 0; i < C; ++i)
      if (cls[i]->c->stream != order) {
        KC_TRY_HIP(hipEventRecord(join[i], cls[i]->c->stream));
        KC_TRY_HIP(hipStreamWaitEvent(order, join[i], 0));
      }
  };
  for (int i = 0; i < C; ++i) {
    ParaClass& pc = *cls[i];
    pc.index = i + 1;
    pc.st.alloc(pc.M, pc.p.max_iter, want_hist);
  }
  int rc_fine = KC_OK;   // a persistent launch left a system above its target
  PersistPlan plan;
  bool use_plan = false;
  if (persistent) {
    std::vector<PersistSpec> specs;
    for (auto* pc : cls) {
      if (!persistent_eligible(pc->p)) continue;
      const int64_t S = (int64_t)pc->p.N * n_unknowns(pc->p);
      double* Fv = (double*)pc->c->ws.get(WS_FINE, sizeof(double) * pc->M * S);
      specs.push_back(PersistSpec{pc->p, pc->a, pc->U, pc->u0, pc->st.active, Fv, pc->M,
                                  tuning_for(pc->c, pc->p.n).fine_pcg_rtol});
      pc->fine_external = true;
    }
    if (!specs.empty()) {
      plan = persistent_prepare(ctx, specs);
      use_plan = true;
    }
  }
  // the persistent fine launch of an iteration (iteration index k: slice 0 only at k = 0)
  auto persist_eager = [&](int k) {
    if (!use_plan) return;
    const DevStatus ds = status_block(ctx);
    status_reset(ctx, ds);
    persistent_launch(ctx, order, plan, k > 0 ? 1 : 0);
    if (status_collect(ctx, ds, 0)) rc_fine = KC_ENOCONV;
  };
  fork_all();
  for (auto* pc : cls) {
    class_init_kernel<<<blocks_of(pc->M), 256, 0, pc->c->stream>>>(pc->M, pc->st.active, pc->st.its, pc->st.status,
                                                                   pc->st.maxima);
    KC_LAUNCH_CHECK();
    if (pc->st.hist)
      zero_kernel<<<blocks_of(pc->M * pc->p.max_iter), 256, 0, pc->c->stream>>>(pc->st.hist,
                                                                               pc->M * pc->p.max_iter);
    KC_LAUNCH_CHECK();
  }
  join_all();
  int rc = KC_OK;
  int k = 0;
  auto read_counts = [&]() {
    KC_TRY_HIP(hipMemcpyAsync(hc.data(), counts, sizeof(int) * (C + 1), hipMemcpyDeviceToHost, order));
    KC_TRY_HIP(hipStreamSynchronize(order));
  };
  // Classes whose iteration is a fixed sequence of launches are captured; a class whose fine
  // sweep steers its own loops from the host (the streamed multigrid path) runs eagerly on
  // its stream beside each replay.
  std::vector<char> in_graph(C, 0);
  int n_graph = 0;
  for (int i = 0; i < C; ++i) {
    in_graph[i] = iteration_capturable(*cls[i]);
    n_graph += in_graph[i];
  }
  // eager iterations (all of them without a graph; the first one with a graph)
  while (k < max_iter) {
    persist_eager(k);
    fork_all();
    for (int i = 0; i < C; ++i)
      if (hc[i + 1] > 0) enqueue_iteration(*cls[i], k, counts, rc);
    join_all();
    read_counts();
    ++k;
    report(k, hc[0]);
    if (hc[0] == 0 || (use_graph && n_graph > 0)) break;
  }
  const bool replay = use_graph && hc[0] > 0 && k < max_iter && n_graph > 0;
  if (replay) {
    // the replays accumulate solver counters into status blocks cleared here
    for (int i = 0; i < C; ++i)
      if (in_graph[i]) {
        status_reset(cls[i]->c, status_block(cls[i]->c, WS_STATUS));
        status_reset(cls[i]->c, status_block(cls[i]->c, WS_STATUS_CGC));
      }
    if (use_plan) {
      status_reset(ctx, status_block(ctx));
      KC_TRY_HIP(hipStreamSynchronize(main));
    }
    for (auto* pc : cls)
      if (pc->c->stream != main) KC_TRY_HIP(hipStreamSynchronize(pc->c->stream));
  }
  if (replay) {
    // capture one iteration of every class (iteration index >= 1: the first slice's
    // fine propagation is not repeated), one branch per class
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t g0, g1;
    KC_TRY_HIP(hipEventCreate(&g0));
    EvGuard g0g{&g0};
    KC_TRY_HIP(hipEventCreate(&g1));
    EvGuard g1g{&g1};
    struct StreamGuard {
      hipStream_t s = nullptr;
      ~StreamGuard() {
        if (s) {
          (void)hipStreamSynchronize(s);
          (void)hipStreamDestroy(s);
        }
      }
    } cs;
    KC_TRY_HIP(hipStreamCreateWithFlags(&cs.s, hipStreamNonBlocking));
    KC_TRY_HIP(hipEventRecord(g0, main));
    KC_TRY_HIP(hipStreamWaitEvent(cs.s, g0, 0));
    order = cs.s;
    KC_TRY_HIP(hipStreamBeginCapture(order, hipStreamCaptureModeRelaxed));
    for (int i = 0; i < C; ++i) cls[i]->c->capturing = in_graph[i] != 0;
    ctx->capturing = use_plan;
    try {
      if (use_plan) persistent_launch(ctx, order, plan, 1);
      KC_TRY_HIP(hipEventRecord(fork, order));
      for (int i = 0; i < C; ++i)
        if (in_graph[i]) {
          if (cls[i]->c->stream != order) KC_TRY_HIP(hipStreamWaitEvent(cls[i]->c->stream, fork, 0));
          enqueue_iteration(*cls[i], 1, counts, rc);
          if (cls[i]->c->stream != order) {
            KC_TRY_HIP(hipEventRecord(join[i], cls[i]->c->stream));
            KC_TRY_HIP(hipStreamWaitEvent(order, join[i], 0));
          }
        }
    } catch (...) {
      for (auto* pc : cls) pc->c->capturing = false;
      ctx->capturing = false;
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(order, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    for (auto* pc : cls) pc->c->capturing = false;
    ctx->capturing = false;
    KC_TRY_HIP(hipStreamEndCapture(order, &graph));
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
      (void)hipGraphDestroy(graph);
      throw Error{KC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie)};
    }
    KC_TRY_HIP(hipEventRecord(g1, order));
    try {
      while (k < max_iter && hc[0] > 0) {
        KC_TRY_HIP(hipGraphLaunch(exec, order));
        for (int i = 0; i < C; ++i)   // the eager classes beside the replay, each on its stream
          if (!in_graph[i] && hc[i + 1] > 0) {
            enqueue_iteration(*cls[i], k, counts, rc);
            KC_TRY_HIP(hipEventRecord(join[i], cls[i]->c->stream));
            KC_TRY_HIP(hipStreamWaitEvent(order, join[i], 0));
          }
        read_counts();
        ++k;
        report(k, hc[0]);
      }
    } catch (...) {
      (void)hipGraphExecDestroy(exec);
      (void)hipGraphDestroy(graph);
      throw;
    }
    float gms = 0.f;
    (void)hipEventElapsedTime(&gms, g0, g1);
    out.graph_ms = gms;
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    // the caller's stream resumes after the replays
    KC_TRY_HIP(hipEventRecord(g1, order));
    KC_TRY_HIP(hipStreamWaitEvent(main, g1, 0));
    order = main;
  }
  out.iterations = k;
  if (replay && use_plan && status_collect(ctx, status_block(ctx), 0)) rc_fine = KC_ENOCONV;
  if (rc == KC_OK) rc = rc_fine;
  if (replay)
    for (int i = 0; i < C; ++i) {   // eager classes collected their counters call by call
      if (!in_graph[i]) continue;
      ParaClass* pc = cls[i];
      if (status_collect(pc->c, status_block(pc->c, WS_STATUS), 0)) rc = KC_ENOCONV;
      if (pc->p.dim == 2 && status_collect(pc->c, status_block(pc->c, WS_STATUS_CGC), 4)) rc = KC_ENOCONV;
    }
  // solver counters and kernel times of the class contexts
  for (auto* pc : cls) {
    const bool own = pc->c != ctx;
    if (!own) continue;
    for (int i = 0; i < 16; ++i) ctx->stats[i] += pc->c->stats[i];
    for (int i = 0; i < 8; ++i) {
      ctx->ktime[i] += pc->c->ktime[i];
      ctx->kcount[i] += pc->c->kcount[i];
    }
  }
  // results
  out.its.clear();
  out.status.clear();
  out.tconv.clear();
  out.hist.clear();
  for (auto* pc : cls) {
    const size_t o = out.its.size();
    out.its.resize(o + pc->M);
    out.status.resize(o + pc->M);
    out.tconv.resize(o + pc->M);
    KC_TRY_HIP(hipMemcpyAsync(&out.its[o], pc->st.its, sizeof(int32_t) * pc->M, hipMemcpyDeviceToHost, main));
    KC_TRY_HIP(hipMemcpyAsync(&out.status[o], pc->st.status, sizeof(int32_t) * pc->M, hipMemcpyDeviceToHost, main));
    KC_TRY_HIP(hipMemcpyAsync(&out.tconv[o], pc->st.tconv, sizeof(unsigned long long) * pc->M,
                              hipMemcpyDeviceToHost, main));
    if (want_hist) {
      const size_t oh = out.hist.size();
      out.hist.resize(oh + (size_t)pc->M * pc->p.max_iter);
      KC_TRY_HIP(hipMemcpyAsync(&out.hist[oh], pc->st.hist, sizeof(double) * pc->M * pc->p.max_iter,
                                hipMemcpyDeviceToHost, main));
    }
  }
  KC_TRY_HIP(hipMemcpyAsync(&out.t0, t0dev, sizeof(unsigned long long), hipMemcpyDeviceToHost, main));
  KC_TRY_HIP(hipStreamSynchronize(main));
  return rc;
}

// Ragged batches: the classes advance independently, each on its own host thread and
// stream.  A class whose iteration is a fixed launch sequence runs its first iteration
// eagerly, then captures one iteration into a graph of its own and replays it; a class whose
// fine sweep steers its loops from the host runs every iteration eagerly.  A class stops as
// soon as all its samples have retired, so the samples of fast classes leave early instead of
// waiting for the slowest class at every iteration.  init_class puts the class's initial
// guess into its U (on the class's stream).
static int run_classes_threads(klecgc_ctx* ctx, std::vector<ParaClass*>& cls, bool use_graph, bool progress,
                               const std::function<int(ParaClass&)>& init_class, DriverOut& out) {
  hipStream_t main = ctx->stream;
  const int C = (int)cls.size();
  char* cbuf = (char*)ctx->ws.get(WS_SMALL, 256 + sizeof(int) * (C + 1));
  unsigned long long* t0dev = (unsigned long long*)cbuf;
  int* counts = (int*)(cbuf + 256);
  std::vector<int> hc(C + 1);
  hc[0] = 0;
  for (int i = 0; i < C; ++i) {
    hc[i + 1] = (int)cls[i]->M;
    hc[0] += hc[i + 1];
  }
  KC_TRY_HIP(hipMemcpyAsync(counts, hc.data(), sizeof(int) * (C + 1), hipMemcpyHostToDevice, main));
  stamp_kernel<<<1, 64, 0, main>>>(t0dev);
  KC_LAUNCH_CHECK();
  hipEvent_t fork = nullptr;
  KC_TRY_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t e;
    ~EvGuard() {
      if (e) (void)hipEventDestroy(e);
    }
  } fg{fork};
  KC_TRY_HIP(hipEventRecord(fork, main));
  std::vector<int> rcs(C, KC_OK), iters(C, 0);
  std::vector<std::exception_ptr> errs(C);
  std::mutex capture_mu;   // one capture at a time
  // Every class sizes its workspace in its first iteration, and growing a workspace frees a
  // buffer, which synchronises the device; that is not allowed while another thread's stream is
  // being captured.  So no class captures before every class has finished its first iteration;
  // until then a class that could capture keeps iterating eagerly instead of waiting.
  std::mutex bar_mu;
  int bar_left = C;
  auto arrive = [&]() {
    std::lock_guard<std::mutex> lk(bar_mu);
    --bar_left;
  };
  auto all_sized = [&]() {
    std::lock_guard<std::mutex> lk(bar_mu);
    return bar_left == 0;
  };
  auto work = [&](int i) {
    ParaClass& pc = *cls[i];
    klecgc_ctx* c = pc.c;
    hipStream_t s = c->stream;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool arrived = false;
    try {
      KC_TRY_HIP(hipSetDevice(ctx->device));
      KC_TRY_HIP(hipStreamWaitEvent(s, fork, 0));
      pc.index = i + 1;
      pc.st.alloc(pc.M, pc.p.max_iter, false);
      class_init_kernel<<<blocks_of(pc.M), 256, 0, s>>>(pc.M, pc.st.active, pc.st.its, pc.st.status, pc.st.maxima);
      KC_LAUNCH_CHECK();
      int r = init_class(pc);
      if (r != KC_OK) rcs[i] = r;
      const bool capture = use_graph && iteration_capturable(pc);
      int left = (int)pc.M, k = 0;
      double last_line = 0.0;
      while (k < pc.p.max_iter && left > 0) {
        if (k == 1 && !arrived) {
          arrived = true;
          arrive();
        }
        if (capture && k >= 1 && !exec && all_sized()) {
          // replays accumulate the solver counters into status blocks cleared here
          status_reset(c, status_block(c, WS_STATUS));
          status_reset(c, status_block(c, WS_STATUS_CGC));
          std::lock_guard<std::mutex> lock(capture_mu);
          KC_TRY_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
          c->capturing = true;
          try {
            enqueue_iteration(pc, 1, counts, rcs[i]);
          } catch (...) {
            c->capturing = false;
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(s, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
          }
          c->capturing = false;
          KC_TRY_HIP(hipStreamEndCapture(s, &graph));
          const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
          if (ie != hipSuccess) throw Error{KC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie)};
        }
        if (exec)
          KC_TRY_HIP(hipGraphLaunch(exec, s));
        else
          enqueue_iteration(pc, k, counts, rcs[i]);
        int hv = 0;
        KC_TRY_HIP(hipMemcpyAsync(&hv, counts + i + 1, sizeof(int), hipMemcpyDeviceToHost, s));
        KC_TRY_HIP(hipStreamSynchronize(s));
        left = hv;
        ++k;
        if (progress || progress_due(last_line))   // every iteration when asked, else one line per 10 s
          std::fprintf(stderr, "[klecgc] class %dx%d N=%d (%lld samples): iteration %d, %d active\n", pc.p.n, pc.p.n,
                       pc.p.N, (long long)pc.M, k, left),
              std::fflush(stderr);
      }
      if (exec) {
        if (status_collect(c, status_block(c, WS_STATUS), 0)) rcs[i] = KC_ENOCONV;
        if (pc.p.dim == 2 && status_collect(c, status_block(c, WS_STATUS_CGC), 4)) rcs[i] = KC_ENOCONV;
      }
      iters[i] = k;
    } catch (...) {
      errs[i] = std::current_exception();
    }
    if (!arrived) arrive();
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  };
  {
    std::vector<std::thread> threads;
    for (int i = 0; i < C; ++i) threads.emplace_back(work, i);
    for (auto& t : threads) t.join();
  }
  for (auto& e : errs)
    if (e) std::rethrow_exception(e);
  int rc = KC_OK;
  for (int r : rcs)
    if (r != KC_OK) rc = r;
  out.iterations = *std::max_element(iters.begin(), iters.end());
  for (auto* pc : cls) {
    for (int i = 0; i < 16; ++i) ctx->stats[i] += pc->c->stats[i];
    for (int i = 0; i < 8; ++i) {
      ctx->ktime[i] += pc->c->ktime[i];
      ctx->kcount[i] += pc->c->kcount[i];
    }
  }
  out.its.clear();
  out.status.clear();
  out.tconv.clear();
  for (auto* pc : cls) {
    const size_t o = out.its.size();
    out.its.resize(o + pc->M);
    out.status.resize(o + pc->M);
    out.tconv.resize(o + pc->M);
    KC_TRY_HIP(hipMemcpyAsync(&out.its[o], pc->st.its, sizeof(int32_t) * pc->M, hipMemcpyDeviceToHost, main));
    KC_TRY_HIP(hipMemcpyAsync(&out.status[o], pc->st.status, sizeof(int32_t) * pc->M, hipMemcpyDeviceToHost, main));
    KC_TRY_HIP(hipMemcpyAsync(&out.tconv[o], pc->st.tconv, sizeof(unsigned long long) * pc->M,
                              hipMemcpyDeviceToHost, main));
  }
  KC_TRY_HIP(hipMemcpyAsync(&out.t0, t0dev, sizeof(unsigned long long), hipMemcpyDeviceToHost, main));
  KC_TRY_HIP(hipStreamSynchronize(main));
  return rc;
}

// ---------------------------------------------------------------- uniform batch
namespace {
// the restricted grid nc of a network whose n_out is N nc^2 (0 if there is none)
int mlp_coarse_grid(const klecgc_mlp* h, int N) {
  const int64_t per = mlp_out_count(h) / N;
  if (per * N != mlp_out_count(h)) return 0;
  int nc = (int)std::llround(std::sqrt((double)per));
  return (int64_t)nc * nc == per ? nc : 0;
}
}  // namespace

// The initial guess U^0 of init mode g.init into U; `used` receives the guess each sample
// started from.  With KC_INIT_MLP_GPC_FALLBACK the fine sweep of iteration 0 is left in the
// WS_FINE buffer and fine_ready is set.
static int initial_guess(klecgc_ctx* ctx, const klecgc_problem& p, const double* a, const double* u0, int64_t M,
                         const GuessArgs& g, double* U, std::vector<int32_t>& used, bool& fine_ready) {
  hipStream_t st = ctx->stream;
  const int64_t Nx = n_unknowns(p);
  const int64_t S = (int64_t)p.N * Nx;
  const int K = p.N / 2 + 1;
  int rc = KC_OK;
  fine_ready = false;
  used.assign(M, g.init);
  auto need_gpc = [&] {
    KC_REQUIRE(g.gpc && g.xi, KC_EINVAL, "gpc handle and xi_dev required for the gPC guess");
    KC_REQUIRE(g.gpc->L == S, KC_EINVAL, "gpc surrogate state length differs from N*Nx");
  };
  auto mlp_guess = [&](double* out) {
    KC_REQUIRE(g.mlp && g.xi, KC_EINVAL, "mlp handle and xi_dev required for the learned guess");
    KC_REQUIRE(p.dim == 2, KC_EUNSUPPORTED, "the learned guess restricts 2D states");
    const int nc = mlp_coarse_grid(g.mlp, p.N);
    KC_REQUIRE(nc > 0, KC_EINVAL, "MLP output size must be N nc^2");
    const int r = mlp_initial_guess_impl(ctx, g.mlp, p.n, nc, p.N, g.xi, M, out);
    if (r != KC_OK) rc = r;
  };
  switch (g.init) {
    case KC_INIT_GIVEN:
      KC_REQUIRE(g.given, KC_EINVAL, "init_dev required for KC_INIT_GIVEN");
      if (g.given != U)
        KC_TRY_HIP(hipMemcpyAsync(U, g.given, sizeof(double) * M * S, hipMemcpyDeviceToDevice, st));
      break;
    case KC_INIT_ZERO:
      KC_TRY_HIP(hipMemsetAsync(U, 0, sizeof(double) * M * S, st));
      break;
    case KC_INIT_COARSE: {
      int r = coarse_sweep_impl(ctx, p, a, u0, M, U);
      if (r != KC_OK) rc = r;
      break;
    }
    case KC_INIT_GPC:
      need_gpc();
      gpc_predict_impl(ctx, g.gpc, g.xi, M, U);
      break;
    case KC_INIT_RANDOM:
      random_guess_kernel<<<blocks_of(M * S, 16384), 256, 0, st>>>((unsigned long long)g.seed, M * S, U);
      KC_LAUNCH_CHECK();
      break;
    case KC_INIT_MLP:
      mlp_guess(U);
      break;
    case KC_INIT_MLP_GPC_FALLBACK: {
      need_gpc();
      mlp_guess(U);
      // the gPC guess and its fine sweep live in the defect and spectrum buffers of the
      // iteration (sized as the iteration asks for them), free until iteration 0's defect
      double* Fv = (double*)ctx->ws.get(WS_FINE, sizeof(double) * M * S);
      double* Ug = (double*)ctx->ws.get(WS_DEFECT, sizeof(double) * M * S);
      double* Fg = (double*)ctx->ws.get(WS_SPEC, sizeof(double) * 2 * M * K * Nx);
      gpc_predict_impl(ctx, g.gpc, g.xi, M, Ug);
      for (int which = 0; which < 2; ++which) {
        FineArgs fa{a, which ? Ug : U, u0, true, 0, nullptr, which ? Fg : Fv, M};
        const int r = fine_propagate_impl(ctx, p, fa);
        if (r != KC_OK) rc = r;
      }
      char* gb = (char*)ctx->ws.get(WS_GUESS, sizeof(unsigned long long) * 4 * M + sizeof(int32_t) * M);
      unsigned long long* mx = (unsigned long long*)gb;
      int32_t* use = (int32_t*)(gb + sizeof(unsigned long long) * 4 * M);
      KC_TRY_HIP(hipMemsetAsync(mx, 0, sizeof(unsigned long long) * 4 * M, st));
      for (int64_t m0 = 0; m0 < M; m0 += 65535) {
        const int64_t Mc = std::min<int64_t>(65535, M - m0);
        guess_defect_kernel<<<dim3(blocks_of(S, 64), (unsigned)Mc), 256, 0, st>>>(
            Fv + m0 * S, U + m0 * S, Fg + m0 * S, Ug + m0 * S, S, mx + 4 * m0);
        KC_LAUNCH_CHECK();
      }
      guess_choose_kernel<<<blocks_of(M), 256, 0, st>>>(mx, M, use);
      KC_LAUNCH_CHECK();
      for (int64_t m0 = 0; m0 < M; m0 += 65535) {
        const int64_t Mc = std::min<int64_t>(65535, M - m0);
        guess_take_kernel<<<dim3(blocks_of(S, 64), (unsigned)Mc), 256, 0, st>>>(use + m0, Ug + m0 * S,
                                                                                Fg + m0 * S, S, U + m0 * S,
                                                                                Fv + m0 * S);
        KC_LAUNCH_CHECK();
      }
      std::vector<int32_t> hu(M);
      KC_TRY_HIP(hipMemcpyAsync(hu.data(), use, sizeof(int32_t) * M, hipMemcpyDeviceToHost, st));
      KC_TRY_HIP(hipStreamSynchronize(st));
      for (int64_t m = 0; m < M; ++m) used[m] = hu[m] ? KC_INIT_GPC : KC_INIT_MLP;
      fine_ready = true;
      break;
    }
    default:
      throw Error{KC_EINVAL, "unknown init mode"};
  }
  return rc;
}

void launch_random_guess(hipStream_t st, uint64_t seed, int64_t n, double* U) {
  random_guess_kernel<<<blocks_of(n, 16384), 256, 0, st>>>((unsigned long long)seed, n, U);
  KC_LAUNCH_CHECK();
}

int parareal_impl(klecgc_ctx* ctx, const klecgc_problem& p, const double* a, const double* u0, int64_t M,
                  const GuessArgs& g, double* U, int32_t* iters, int32_t* status, double* hist, int32_t* guess) {
  bool fine_ready = false;
  std::vector<int32_t> used;
  int rc = initial_guess(ctx, p, a, u0, M, g, U, used, fine_ready);
  ParaClass pc;
  pc.c = ctx;
  pc.p = p;
  pc.pb = p;
  // The parareal loop solves the coarse system for the correction U^{k+1} - U^k, whose
  // right-hand side is the defect; errors of the shifted solves then only perturb the
  // contraction (by ~ cgc_rtol / alpha), not the fixed point, so a relative 1e-7
  // suffices by default.
  if (pc.pb.cgc_rtol <= 0) pc.pb.cgc_rtol = 1e-7;
  pc.M = M;
  pc.a = a;
  pc.u0 = u0;
  pc.U = U;
  pc.fine_ready = fine_ready;
  std::vector<ParaClass*> cls{&pc};
  DriverOut out;
  int r = run_classes(ctx, cls, false, hist != nullptr, out);
  if (r != KC_OK) rc = r;
  std::memcpy(iters, out.its.data(), sizeof(int32_t) * M);
  std::memcpy(status, out.status.data(), sizeof(int32_t) * M);
  if (hist) std::memcpy(hist, out.hist.data(), sizeof(double) * M * p.max_iter);
  if (guess) std::memcpy(guess, used.data(), sizeof(int32_t) * M);
  return rc;
}

// ---------------------------------------------------------------- Algorithm 1
namespace {
// D = F - G of the old starts; Unew[m][0] = F[m][0] (G(u0) cancels)
// (Gv and D may be the same buffer: each element is read before it is written)
__global__ void seq_diff_kernel(const double* __restrict__ Fv, const double* Gv,
                                const uint8_t* __restrict__ active, int64_t S, int64_t Nx, double* D,
                                double* __restrict__ Unew) {
  const int64_t m = blockIdx.y;
  if (!active[m]) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S; i += (int64_t)gridDim.x * blockDim.x) {
    const double f = Fv[m * S + i];
    D[m * S + i] = f - Gv[m * S + i];
    if (i < Nx) Unew[m * S + i] = f;
  }
}

// Unew[m][s] = G(Unew[m][s-1]) + D[m][s] with the coarse step's result g [M][Nx]
__global__ void seq_correct_kernel(const double* __restrict__ g, const double* __restrict__ D,
                                   const uint8_t* __restrict__ active, int64_t S, int64_t Nx, int s,
                                   double* __restrict__ Unew) {
  const int64_t m = blockIdx.y;
  if (!active[m]) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < Nx; i += (int64_t)gridDim.x * blockDim.x)
    Unew[m * S + (int64_t)s * Nx + i] = g[m * Nx + i] + D[m * S + (int64_t)s * Nx + i];
}

// maxima[2m] = max |Unew - U|, maxima[2m+1] = max |Unew| (ordered bit patterns); U = Unew
__global__ __launch_bounds__(256) void seq_increment_kernel(const double* __restrict__ Unew,
                                                            const uint8_t* __restrict__ active, int64_t S,
                                                            double* __restrict__ U,
                                                            unsigned long long* __restrict__ maxima) {
  const int64_t m = blockIdx.y;
  if (!active[m]) return;
  double c = 0.0, u = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < S; i += (int64_t)gridDim.x * blockDim.x) {
    const double nv = Unew[m * S + i];
    c = nanmax(c, fabs(nv - U[m * S + i]));
    u = nanmax(u, fabs(nv));
    U[m * S + i] = nv;
  }
  c = wave_nanmax(c);
  u = wave_nanmax(u);
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&maxima[2 * m], (unsigned long long)__double_as_longlong(c));
    atomicMax(&maxima[2 * m + 1], (unsigned long long)__double_as_longlong(u));
  }
}
}  // namespace

int parareal_seq_impl(klecgc_ctx* ctx, const klecgc_problem& p, const double* a, const double* u0, int64_t M,
                      const GuessArgs& g, double* U, int32_t* iters, int32_t* status, double* hist) {
  KC_REQUIRE(g.init != KC_INIT_MLP_GPC_FALLBACK, KC_EUNSUPPORTED,
             "the sequential coarse grid correction takes a single initial guess");
  hipStream_t st = ctx->stream;
  const int64_t Nx = n_unknowns(p);
  const int64_t S = (int64_t)p.N * Nx;
  bool fine_ready = false;
  std::vector<int32_t> used;
  int rc = initial_guess(ctx, p, a, u0, M, g, U, used, fine_ready);
  double* Fv = (double*)ctx->ws.get(WS_FINE, sizeof(double) * M * S);
  double* D = (double*)ctx->ws.get(WS_DEFECT, sizeof(double) * M * S);
  double* Un = (double*)ctx->ws.get(WS_SPEC, sizeof(double) * M * S);
  double* stage = (double*)ctx->ws.get(WS_START, sizeof(double) * Nx * M);
  double* gout = (double*)ctx->ws.get(WS_GEMM_A, sizeof(double) * Nx * M);
  int* counts = (int*)ctx->ws.get(WS_SMALL, sizeof(int) * 2);
  ClassState cs;
  cs.alloc(M, p.max_iter, hist != nullptr);
  class_init_kernel<<<blocks_of(M), 256, 0, st>>>(M, cs.active, cs.its, cs.status, cs.maxima);
  KC_LAUNCH_CHECK();
  if (cs.hist) {
    zero_kernel<<<blocks_of(M * p.max_iter), 256, 0, st>>>(cs.hist, M * p.max_iter);
    KC_LAUNCH_CHECK();
  }
  int hc[2] = {(int)M, (int)M};
  KC_TRY_HIP(hipMemcpyAsync(counts, hc, sizeof(hc), hipMemcpyHostToDevice, st));
  const double dT = p.T / p.N;
  const dim3 gs(blocks_of(S, 64), (unsigned)M);
  const dim3 gx(blocks_of(Nx, 64), (unsigned)M);
  for (int k = 0; k < p.max_iter; ++k) {
    // F and G of the old starts u0, U_0 .. U_{N-2}, all slices at once (F(u0) once)
    FineArgs ff{a, U, u0, true, k > 0 ? 1 : 0, cs.active, Fv, M};
    int r = fine_propagate_impl(ctx, p, ff);
    if (r != KC_OK) rc = r;
    FineArgs fg{a, U, u0, true, 0, cs.active, D, M};
    r = propagate_impl(ctx, p, fg, dT, 1, p.N);   // G of the old starts, into D
    if (r != KC_OK) rc = r;
    seq_diff_kernel<<<gs, 256, 0, st>>>(Fv, D, cs.active, S, Nx, D, Un);
    KC_LAUNCH_CHECK();
    // the correction sweeps the slices: U^{k+1}_s = G(U^{k+1}_{s-1}) + F_s - G_s
    for (int s = 1; s < p.N; ++s) {
      KC_TRY_HIP(hipMemcpy2DAsync(stage, sizeof(double) * Nx, Un + (int64_t)(s - 1) * Nx, sizeof(double) * S,
                                  sizeof(double) * Nx, M, hipMemcpyDeviceToDevice, st));
      FineArgs fc{a, stage, nullptr, false, 0, cs.active, gout, M};
      r = propagate_impl(ctx, p, fc, dT, 1, 1);
      if (r != KC_OK) rc = r;
      seq_correct_kernel<<<gx, 256, 0, st>>>(gout, D, cs.active, S, Nx, s, Un);
      KC_LAUNCH_CHECK();
    }
    seq_increment_kernel<<<gs, 256, 0, st>>>(Un, cs.active, S, U, cs.maxima);
    KC_LAUNCH_CHECK();
    converge_kernel<<<blocks_of(M), 256, 0, st>>>(M, p.max_iter, p.tol, cs.maxima, cs.active, cs.its, cs.status,
                                                  cs.hist, nullptr, counts, 1);
    KC_LAUNCH_CHECK();
    KC_TRY_HIP(hipMemcpyAsync(hc, counts, sizeof(hc), hipMemcpyDeviceToHost, st));
    KC_TRY_HIP(hipStreamSynchronize(st));
    if (hc[0] == 0) break;
  }
  KC_TRY_HIP(hipMemcpyAsync(iters, cs.its, sizeof(int32_t) * M, hipMemcpyDeviceToHost, st));
  KC_TRY_HIP(hipMemcpyAsync(status, cs.status, sizeof(int32_t) * M, hipMemcpyDeviceToHost, st));
  if (hist) KC_TRY_HIP(hipMemcpyAsync(hist, cs.hist, sizeof(double) * M * p.max_iter, hipMemcpyDeviceToHost, st));
  KC_TRY_HIP(hipStreamSynchronize(st));
  return rc;
}

// ---------------------------------------------------------------- ragged batch
namespace {
struct SubCtx {
  klecgc_ctx c;
  SubCtx(int device, int num_cus) {
    c.device = device;
    c.num_cus = num_cus;
    KC_TRY_HIP(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
    KC_TRY_HIP(hipEventCreate(&c.ev[0]));
    KC_TRY_HIP(hipEventCreate(&c.ev[1]));
  }
  ~SubCtx() {
    if (c.stream) (void)hipStreamSynchronize(c.stream);
    c.ws.release();
    for (auto& e : c.ev)
      if (e) (void)hipEventDestroy(e);
    if (c.stream) (void)hipStreamDestroy(c.stream);
  }
};
}  // namespace

int parareal_batch_impl(klecgc_ctx* ctx, const klecgc_problem& base, const klecgc_task* tasks, int64_t M,
                        const double* a, int32_t init, double* U, int32_t flags, int32_t* iters, int32_t* status,
                        double* latency_ms, double* total_ms) {
  KC_REQUIRE(init == KC_INIT_ZERO || init == KC_INIT_COARSE || init == KC_INIT_GIVEN, KC_EUNSUPPORTED,
             "parareal_solve_batch supports KC_INIT_ZERO, KC_INIT_COARSE and KC_INIT_GIVEN");
  hipStream_t main = ctx->stream;
  // classes of equal (n, N), largest estimated cost first
  std::map<std::pair<int, int>, std::vector<int64_t>> groups;
  for (int64_t m = 0; m < M; ++m) {
    const klecgc_task& t = tasks[m];
    KC_REQUIRE(t.face_off >= 0 && t.state_off >= 0, KC_EINVAL, "task offsets must be >= 0");
    klecgc_problem q = base;
    q.n = t.n;
    q.N = t.N;
    validate_problem(q);
    groups[{t.n, t.N}].push_back(m);
  }
  std::vector<std::pair<std::pair<int, int>, std::vector<int64_t>>> order(groups.begin(), groups.end());
  auto cost = [&](const std::pair<int, int>& k) {
    const double nn = base.dim == 1 ? k.first : (double)k.first * k.first;
    return nn * k.second * (base.dim == 1 ? 1.0 : k.first);  // ~ unknowns x slices x Krylov its
  };
  std::stable_sort(order.begin(), order.end(), [&](const auto& x, const auto& y) {
    return cost(x.first) * x.second.size() > cost(y.first) * y.second.size();
  });
  const int C = (int)order.size();
  std::vector<std::unique_ptr<SubCtx>> subs;
  std::vector<std::unique_ptr<ParaClass>> pcs;
  struct Bufs {
    void* p = nullptr;
    ~Bufs() {
      if (p) (void)hipFree(p);
    }
  };
  std::vector<std::unique_ptr<Bufs>> bufs;
  hipEvent_t e0, e1;
  KC_TRY_HIP(hipEventCreate(&e0));
  KC_TRY_HIP(hipEventCreate(&e1));
  struct EvPair {
    hipEvent_t a, b;
    ~EvPair() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } evp{e0, e1};
  KC_TRY_HIP(hipEventRecord(e0, main));
  int rc = KC_OK;
  for (int i = 0; i < C; ++i) {
    const auto& key = order[i].first;
    const auto& idx = order[i].second;
    subs.emplace_back(new SubCtx(ctx->device, ctx->num_cus));
    klecgc_ctx* sc = &subs.back()->c;
    sc->tuning = ctx->tuning;
    auto pc = std::make_unique<ParaClass>();
    pc->c = sc;
    pc->p = base;
    pc->p.n = key.first;
    pc->p.N = key.second;
    pc->pb = pc->p;
    if (pc->pb.cgc_rtol <= 0) pc->pb.cgc_rtol = 1e-7;
    const int64_t Mc = (int64_t)idx.size();
    const int64_t Nx = n_unknowns(pc->p), Fc = n_faces(base.dim, key.first);
    const int64_t S = (int64_t)key.second * Nx;
    pc->M = Mc;
    // gather faces (and the given guess) into contiguous class buffers
    bufs.emplace_back(new Bufs);
    const size_t bytes = sizeof(double) * (size_t)Mc * (Fc + S) + 2 * sizeof(int64_t) * Mc + 512;
    if (hipMalloc(&bufs.back()->p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      bufs.back()->p = nullptr;
      throw Error{KC_ENOMEM, "ragged class buffer allocation failed"};
    }
    double* ac = (double*)bufs.back()->p;
    double* Uc = ac + Mc * Fc;
    int64_t* offs = (int64_t*)(((uintptr_t)(Uc + Mc * S) + 255) & ~(uintptr_t)255);
    std::vector<int64_t> ho(2 * Mc);
    for (int64_t j = 0; j < Mc; ++j) {
      ho[j] = tasks[idx[j]].face_off;
      ho[Mc + j] = tasks[idx[j]].state_off;
    }
    KC_TRY_HIP(hipMemcpyAsync(offs, ho.data(), sizeof(int64_t) * 2 * Mc, hipMemcpyHostToDevice, main));
    launch_rows(true, main, a, offs, Fc, Mc, ac);
    if (init == KC_INIT_GIVEN) launch_rows(true, main, U, offs + Mc, S, Mc, Uc);
    pc->a = ac;
    pc->u0 = nullptr;
    pc->U = Uc;
    pcs.push_back(std::move(pc));
  }
  KC_TRY_HIP(hipStreamSynchronize(main));
  std::vector<ParaClass*> cls;
  for (auto& pc : pcs) cls.push_back(pc.get());
  auto init_class = [&](ParaClass& pc) -> int {
    if (init == KC_INIT_ZERO) {
      zero_kernel<<<blocks_of(pc.M * pc.p.N * n_unknowns(pc.p)), 256, 0, pc.c->stream>>>(
          pc.U, pc.M * pc.p.N * n_unknowns(pc.p));
      KC_LAUNCH_CHECK();
    } else if (init == KC_INIT_COARSE) {
      return coarse_sweep_impl(pc.c, pc.p, pc.a, nullptr, pc.M, pc.U);
    }
    return KC_OK;
  };
  DriverOut out;
  int r;
  if (flags & KC_BATCH_PERSISTENT) {
    // one thread, one graph: each iteration is one persistent fine launch over the classes
    // that qualify, then every class's branch (its own fine sweep otherwise, the correction)
    for (auto* pc : cls) {
      const int ri = init_class(*pc);
      if (ri != KC_OK) rc = ri;
    }
    for (auto* pc : cls) KC_TRY_HIP(hipStreamSynchronize(pc->c->stream));
    r = run_classes(ctx, cls, (flags & KC_BATCH_GRAPH) != 0, false, out, (flags & KC_BATCH_PROGRESS) != 0, true);
  } else {
    r = run_classes_threads(ctx, cls, (flags & KC_BATCH_GRAPH) != 0, (flags & KC_BATCH_PROGRESS) != 0, init_class,
                            out);
  }
  if (r != KC_OK) rc = r;
  // scatter the iterates back
  for (int i = 0; i < C; ++i) {
    ParaClass& pc = *pcs[i];
    const int64_t S = (int64_t)pc.p.N * n_unknowns(pc.p);
    const int64_t Fc = n_faces(base.dim, pc.p.n);
    double* Uc = pc.U;
    int64_t* offs = (int64_t*)(((uintptr_t)(Uc + pc.M * S) + 255) & ~(uintptr_t)255);
    (void)Fc;
    launch_rows(false, main, Uc, offs + pc.M, S, pc.M, U);
  }
  KC_TRY_HIP(hipEventRecord(e1, main));
  KC_TRY_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  KC_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
  if (total_ms) *total_ms = ms;
  int rate_khz = 0;
  KC_TRY_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, ctx->device));
  size_t o = 0;
  for (int i = 0; i < C; ++i) {
    for (int64_t j : order[i].second) {
      iters[j] = out.its[o];
      status[j] = out.status[o];
      if (latency_ms) {
        const unsigned long long t = out.tconv[o];
        latency_ms[j] = (t > out.t0 && rate_khz > 0) ? (double)(t - out.t0) / (double)rate_khz : -1.0;
      }
      ++o;
    }
  }
  return rc;
}

}  // namespace kc
