// Internal definitions shared by the KLE-CGC library sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "klecgc.h"

namespace kc {

// ---- error plumbing ---------------------------------------------------------
struct Error {
  int code;
  std::string msg;
};

#define KC_TRY_HIP(expr)                                                                  \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::kc::Error{KC_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)};      \
  } while (0)

#define KC_REQUIRE(cond, code, text)                                                      \
  do {                                                                                    \
    if (!(cond)) throw ::kc::Error{(code), std::string(text)};                            \
  } while (0)

#define KC_LAUNCH_CHECK() KC_TRY_HIP(hipGetLastError())

// ---- device workspace ---------------------------------------------------------
// Grow-only device buffers keyed by slot; freed when the context is destroyed.  In arena
// mode (`arena` set) slots are carved in request order from a fixed region the workspace
// does not own, nothing is allocated or freed, and a request beyond the region throws.
struct Workspace {
  std::vector<void*> ptr;
  std::vector<size_t> cap;
  char* arena = nullptr;
  size_t arena_bytes = 0, arena_used = 0;
  void* get(int slot, size_t bytes);
  size_t arena_left() const { return arena_bytes - arena_used; }
  void release();
};

enum WsSlot {
  WS_FACTORS = 0,   // per-sample solver tables
  WS_FSCALED,       // float32 Jacobi-scaled coefficients
  WS_DINV,          // float64 D^{-1/2}
  WS_KRYLOV,        // streaming Krylov vectors
  WS_FINE,          // parareal: F(U) buffer
  WS_DEFECT,        // parareal: defect buffer
  WS_SPEC,          // spectral (complex) buffer
  WS_SMALL,         // small per-sample arrays (flags, maxima)
  WS_START,         // start buffer for the coarse sweep
  WS_GEMM_A,
  WS_GEMM_B,
  WS_STATUS,        // status block of the fine propagator
  WS_STATUS_CGC,    // status block of the shifted solves
  WS_FINE_AUX,      // float32 correction tiles of the shifted solves
  WS_MLP,           // MLP predictions before prolongation
  WS_FINE_INC,      // fine propagator: per-system increment of the current step
  WS_GUESS,         // parareal: per-sample guess choice (flags, defect maxima)
  WS_MG_COEF,       // streamed multigrid: per-sample coarse operators
  WS_MG_SMALL,      // streamed multigrid: band partials, per-system state, counters
  WS_MODEL_FAC,     // model problems: real step-matrix factors
  WS_MODEL_CFAC,    // model problems: complex shifted-system factors
  WS_MODEL_WORK,    // model problems: per-lane work vectors of the fine sweep
  WS_MODEL_STATE,   // model problems: fine results, defects
  WS_MODEL_SPEC,    // model problems: slice spectra
  WS_MODEL_SMALL,   // model problems: tables, lists, maxima, initial values
  WS_MODEL_AUX,     // model problems: second state buffer (Algorithm 1, Newton)
  WS_PERSIST,       // persistent fine launch: class descriptors, task counters, tables
  WS_COUNT
};

}  // namespace kc

// Kernel choices and inner tolerances for 2D float32-refined problems of one grid size
// (set by the autotuner or klecgc_set_tuning; the defaults are the built-in heuristic).
struct KcTuning {
  int fine_variant = -1;        // -1 heuristic; KC_FINE_* otherwise
  float fine_pcg_rtol = 1e-6f;  // float32 PCG residual reduction per refinement pass
  int cgc_variant = -1;         // -1 heuristic; KC_CGC_* otherwise
  float cgc_inner_rtol = 1e-5f; // float32 COCG residual reduction per refinement pass
  int mg_sweeps = 0;            // multigrid smoothing sweeps per level (0 = default 2)
  int mg_smoother = 0;          // 0 red-black Gauss-Seidel, 1 damped Jacobi
};

struct klecgc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  kc::Workspace ws;
  int num_cus = 256;
  // counters of the last call: [0..3] fine solves (Krylov iterations, refinement passes,
  // implicit steps, max iterations of one solve), [4..7] the same for the shifted solves
  // [8] shader-clock cycles of the fine kernel summed over work-groups, [9] of which in
  // the float32 Krylov loops
  int64_t stats[16] = {0};
  // HIP-event time (ms) and launch count per kernel class of the last call
  double ktime[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t kcount[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  hipEvent_t ev[2] = {nullptr, nullptr};
  void* blas = nullptr;   // rocblas handle of the offline eigen-solver (created on first use)
  // true while the context's launches are being captured into a graph: no event timing,
  // no status resets or read-backs (the parareal loop does them around the captured region)
  bool capturing = false;
  std::map<int, KcTuning> tuning;   // by grid size n
  void* scratch = nullptr;          // this device's copy of the allocation-free scratch array
};

struct klecgc_kle {
  int32_t kind = 0;
  // FIELD_EXP
  int32_t dim = 0, n = 0, d = 0;
  int64_t nfaces = 0;
  double* phi = nullptr;      // [d][Fc] device
  double* sqrt_lam = nullptr; // [d] device
  std::vector<double> lam_host;
  // SNAPSHOT
  int64_t L = 0, n_t = 0;
  int32_t n_modes = 0;
  double* mean = nullptr;     // [L]
  double* W = nullptr;        // [M_Q][L]  rows sqrt(lam_k) g_k
  double* lam = nullptr;      // [M_Q]
  std::vector<double> zeta_train;  // [n_t][M_Q] host (training coefficients)
};

struct klecgc_gpc {
  int32_t d = 0, p = 0, P = 0, n_modes = 0;
  int32_t basis = KC_GPC_HERMITE;
  int64_t L = 0;
  int32_t* idx = nullptr;     // [P][d] device multi-indices
  double* H = nullptr;        // [P][M_Q] device
  const klecgc_kle* kl = nullptr;
  double* mean = nullptr;     // [L] device (copy of the KL mean)
  double* W = nullptr;        // [M_Q][L] device (copy of sqrt(lam) g rows)
};

namespace kc {

// Device status block: int flag at byte 0, unsigned long long counters from byte 8.
constexpr size_t kStatusBytes = 256;
struct DevStatus {
  int* flag;
  unsigned long long* cnt;
};
DevStatus status_block(klecgc_ctx* ctx, int slot = WS_STATUS);
// zeroes the block (no-op while capturing)
void status_reset(klecgc_ctx* ctx, const DevStatus& st);
// copies the block to the host, adds the counters into ctx->stats[base..base+3] (and
// the cycle counters 8, 9 for base 0); returns flag (0 without reading while capturing)
int status_collect(klecgc_ctx* ctx, const DevStatus& st, int base);

// Kernel classes timed with HIP events on the context stream.
enum KClass { KT_FINE = 0, KT_SHIFTED = 1, KT_FFT_FWD = 2, KT_FFT_INV = 3, KT_DEFECT = 4, KT_GEMM = 5, KT_MLP = 6, KT_COUNT = 8 };
// Records an event pair around `launch` and adds the elapsed time to ctx->ktime[cls]
// (synchronises the stream).
template <class F>
void timed(klecgc_ctx* ctx, int cls, F&& launch) {
  if (ctx->capturing) {
    launch();
    return;
  }
  KC_TRY_HIP(hipEventRecord(ctx->ev[0], ctx->stream));
  launch();
  KC_TRY_HIP(hipEventRecord(ctx->ev[1], ctx->stream));
  KC_TRY_HIP(hipEventSynchronize(ctx->ev[1]));
  float ms = 0.f;
  KC_TRY_HIP(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
  ctx->ktime[cls] += ms;
  ctx->kcount[cls] += 1;
}

inline KcTuning tuning_for(const klecgc_ctx* ctx, int n) {
  auto it = ctx->tuning.find(n);
  return it == ctx->tuning.end() ? KcTuning{} : it->second;
}
// the fine / shifted-solve kernel a 2D float32-refined problem of grid size n runs
int fine_variant_for(int n, int requested);
int cgc_variant_for(int n, int requested);
bool fine_variant_fits(int v, int n);
bool cgc_variant_fits(int v, int n);

inline int64_t n_unknowns(const klecgc_problem& p) { return p.dim == 1 ? p.n : (int64_t)p.n * p.n; }
inline int64_t n_faces(int dim, int n) { return dim == 1 ? n + 1 : 2LL * n * (n + 1); }

void validate_problem(const klecgc_problem& p);

// ---- kernels' host launchers -------------------------------------------------
// field
void launch_field_synth(hipStream_t s, const double* phi, const double* sqrt_lam, int d,
                        int64_t nfaces, const double* xi, int64_t M, double* a, float* a32);
// fine propagator
// start rows: if start_shift, the start of (m, s) is u0[m] (or 0) for s == 0 and
// U[m][s-1] otherwise (the parareal layout); else start[m][s].
struct FineArgs {
  const double* a;
  const double* start;
  const double* u0;       // used with start_shift (nullable = zero)
  bool start_shift;
  int skip_first;         // skip slice 0 (iteration-invariant F(u0))
  const uint8_t* active;  // [M] nullable
  double* out;
  int64_t M;
};
int fine_propagate_impl(klecgc_ctx* ctx, const klecgc_problem& p, const FineArgs& fa);
// The fine sweeps of several parareal classes in one persistent launch (fine.hip).  A class
// qualifies if it is 2D, float32-refined and n <= 128 (it is then solved by the red-black
// resident kernel whatever its tuning says).
struct PersistSpec {
  klecgc_problem p;
  const double* a;          // [M][Fc]
  const double* U;          // iterate [M][N][Nx]: slice s starts from U[m][s-1]
  const double* u0;         // slice 0's start (nullable: zero)
  const uint8_t* active;    // [M] nullable
  double* out;              // F(U) [M][N][Nx]
  int64_t M;
  float pcg_rtol;
};
struct PersistPlan {
  void* cls = nullptr;                 // device descriptors
  int ncls = 0;
  int64_t ntasks = 0;                  // (sample, slice) tasks of all classes
  int nmax = 0;
  int grid = 0;
  double* incbuf = nullptr;
  unsigned long long* queue = nullptr;
};
bool persistent_eligible(const klecgc_problem& p);
// builds every class's tables and the descriptors in ctx's workspace (outside capture)
PersistPlan persistent_prepare(klecgc_ctx* ctx, const std::vector<PersistSpec>& cls);
// one launch on stream st over every task (capturable); counters into ctx's status block
void persistent_launch(klecgc_ctx* ctx, hipStream_t st, const PersistPlan& plan, int skip_first);
// multigrid-preconditioned fine propagation streamed pass by pass (fine_mg.hip); dinv and the
// scaled float32 couplings sf of every sample are built by the caller
int fine_mg_streamed(klecgc_ctx* ctx, const klecgc_problem& p, const FineArgs& fa, double tau, int J, int N,
                     const double* dinv, const float* sf, int* flag, unsigned long long* cnt);

// coarse grid correction pieces
void launch_defect(hipStream_t s, const klecgc_problem& p, const double* a, const double* Fv,
                   const double* U, const uint8_t* active, int64_t M, double* D);
void launch_fft_forward(hipStream_t s, const klecgc_problem& p, const double* r,
                        const uint8_t* active, int64_t M, double* spec);
void launch_fft_inverse(hipStream_t s, const klecgc_problem& p, const double* spec,
                        const uint8_t* active, int64_t M, double* u, bool accumulate,
                        unsigned long long* maxima);
int shifted_solve_impl(klecgc_ctx* ctx, const klecgc_problem& p, const double* a,
                       const uint8_t* active, int64_t M, double* spec);
int coarse_sweep_impl(klecgc_ctx* ctx, const klecgc_problem& p, const double* a,
                      const double* u0, int64_t M, double* U);
int serial_fine_impl(klecgc_ctx* ctx, const klecgc_problem& p, const double* a,
                     const double* u0, int64_t M, double* U);

// dense float64 GEMM: C[m][n] = beta_bias[n] + sum_k A[m][k] B[k][n]  (row-major,
// lda/ldb/ldc leading dimensions); bias nullable.
void launch_dgemm(hipStream_t s, int64_t Mr, int64_t Nc, int64_t K, const double* A, int64_t lda,
                  const double* B, int64_t ldb, double* C, int64_t ldc, const double* bias,
                  double alpha);
// C = alpha * A^T-style products used by the snapshot KL
void launch_dgemm_tn(hipStream_t s, int64_t Mr, int64_t Nc, int64_t K, const double* A,
                     int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                     double alpha);
void launch_gpc_basis(hipStream_t s, const double* xi, int64_t M, int d, const int32_t* idx, int P,
                      int basis, double* Psi);
void launch_col_mean_center(hipStream_t s, const double* S, int64_t n_t, int64_t L, double* mean,
                            double* Sc);

// gPC prediction U0 = mean + Psi(xi) H W (abi.cpp)
int gpc_predict_impl(klecgc_ctx* ctx, const klecgc_gpc* g, const double* xi, int64_t M, double* U0);
// parareal drivers (batch.hip)
// the initial guess of parareal_solve (KC_INIT_*) and what it reads
struct GuessArgs {
  int32_t init;
  const double* given;      // KC_INIT_GIVEN
  const klecgc_gpc* gpc;    // KC_INIT_GPC, KC_INIT_MLP_GPC_FALLBACK
  klecgc_mlp* mlp;          // KC_INIT_MLP, KC_INIT_MLP_GPC_FALLBACK
  const double* xi;         // [M][d] for the surrogates
  uint64_t seed;            // KC_INIT_RANDOM
};
int parareal_impl(klecgc_ctx* ctx, const klecgc_problem& p, const double* a, const double* u0, int64_t M,
                  const GuessArgs& g, double* U, int32_t* iters, int32_t* status, double* hist, int32_t* guess);
int parareal_seq_impl(klecgc_ctx* ctx, const klecgc_problem& p, const double* a, const double* u0, int64_t M,
                      const GuessArgs& g, double* U, int32_t* iters, int32_t* status, double* hist);
// J steps of size tau over N slices per sample (fine propagation with tau = dT/J; one coarse
// step with tau = dT, J = 1)
int propagate_impl(klecgc_ctx* ctx, const klecgc_problem& p, const FineArgs& fa, double tau, int J, int N);
int parareal_batch_impl(klecgc_ctx* ctx, const klecgc_problem& base, const klecgc_task* tasks, int64_t M,
                        const double* a, int32_t init, double* U, int32_t flags, int32_t* iters, int32_t* status,
                        double* latency_ms, double* total_ms);

// autotuner (tune.cpp)
int autotune_impl(klecgc_ctx* ctx, const klecgc_problem& p, const double* a, int64_t M, klecgc_tuning* out,
                  double* ms_out);

// MLP initial guess (BF16 MFMA)
int64_t mlp_param_count(const klecgc_mlp* h);
int64_t mlp_out_count(const klecgc_mlp* h);
int mlp_in_count(const klecgc_mlp* h);
int mlp_create_impl(klecgc_ctx* ctx, int n_in, int hidden, int64_t n_out, klecgc_mlp** out);
int mlp_set_params_impl(klecgc_ctx* ctx, klecgc_mlp* h, const float* params);
int mlp_get_params_impl(klecgc_ctx* ctx, const klecgc_mlp* h, float* params, float* mean, float* stdv);
int mlp_normalize_impl(klecgc_ctx* ctx, klecgc_mlp* h, float* Y, int64_t n);
int mlp_predict_impl(klecgc_ctx* ctx, klecgc_mlp* h, const double* xi, int64_t M, float* Y);
int mlp_grad_impl(klecgc_ctx* ctx, klecgc_mlp* h, const double* xi, const float* Y, int64_t n, float* grads,
                  double* loss);
int mlp_train_impl(klecgc_ctx* ctx, klecgc_mlp* h, const double* xi, const float* Y, int64_t n, int epochs, int batch,
                   float lr, float lr_final, const int32_t* perm, float* loss_host);
int grid_restrict_impl(klecgc_ctx* ctx, int n, int nc, const double* U, int64_t R, float* Yc);
int mlp_initial_guess_impl(klecgc_ctx* ctx, klecgc_mlp* h, int n, int nc, int N, const double* xi, int64_t M,
                           double* U0);

// Progress lines on stderr from long-running loops, enabled by the environment variable
// KLECGC_PROGRESS=1 (read once); `progress_due` rate-limits a loop to one line per 10 s.
bool progress_enabled();
bool progress_due(double& last_s);
void progress_line(const char* fmt, ...);

// the allocation-free scratch array (noalloc.hip): resolves this device's copy (the device
// must be current), its size, and a fill kernel that clears device memory without a memset
hipError_t scratch_resolve(int device, void** out);
size_t scratch_bytes();
void launch_zero_bytes(hipStream_t s, void* p, size_t bytes);

// host linear algebra
// Gram eigen-decomposition on the device (eig.cpp): Cd [n][n] symmetric (overwritten) ->
// V (host, row-major, eigenvectors as columns) and w, descending
void gram_eig(klecgc_ctx* ctx, int n, double* Cd, std::vector<double>& V, std::vector<double>& w);
void release_blas(klecgc_ctx* ctx);
int householder_lstsq(int m, int n, int nrhs, std::vector<double>& B, std::vector<double>& D,
                      std::vector<double>& X);

}  // namespace kc
