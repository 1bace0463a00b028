/*
 * klecgc.h -- C ABI of the MI355X (gfx950) KLE-CGC library.
 *
 * KLE-CGC (arXiv 2510.26180) solves the parametric linear diffusion problem
 *     u' = -A(xi) u + f,  u(0) = u0,  t in [0, T]                  (Section 2, eq. psys;
 *                                                                    Section 4.1, eq. ODE)
 * for many samples xi by parareal with a diagonalised coarse grid correction
 * (Section 3.2, Algorithm 2) started from a KL/gPC initial guess (Algorithm 3).
 *
 * Conventions
 *  - Every `*_dev` pointer is caller-owned device memory on the context's device,
 *    contiguous, row-major, with the layout stated at each argument.  The library
 *    never frees, keeps or reads caller pointers after a call returns (work is
 *    enqueued on the context's stream; a call that writes host memory
 *    synchronises that stream before returning).
 *  - States are [M][N][Nx] float64 with x fastest; in 2D the unknown of node
 *    (i, j) (0-based, x = (i+1)h, y = (j+1)h, h = 1/(n+1)) is j*n + i.
 *  - Face coefficients a are [M][Fc] float64:
 *      1D: Fc = n+1, face f between nodes f-1 and f (nodes -1 and n are the
 *          zero-Dirichlet boundary), at x = (f + 1/2) h;
 *      2D: Fc = 2n(n+1); x-faces first, index j*(n+1)+f between nodes (f-1, j)
 *          and (f, j); then y-faces, index n(n+1) + f*n + i between (i, f-1) and
 *          (i, f).
 *    The operator is (A u)_p = sum over the faces of p of a_f (u_p - u_q) / h^2
 *    with u_q = 0 outside the grid.
 *  - Library-owned handles are created by kle_build / gpc_fit and released
 *    with klecgc_kle_free / klecgc_gpc_free.
 *  - Errors: every entry point returns KC_OK or a negative code; no exception
 *    or abort crosses the ABI.  klecgc_last_error(ctx) returns a message for
 *    the last failing call on that context (valid until the next call).
 *  - One context per host thread.
 */
#ifndef KLECGC_H
#define KLECGC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  KC_OK = 0,
  KC_EINVAL = -1,        /* invalid argument (null pointer, bad size or parameter) */
  KC_ENOMEM = -2,        /* device or host allocation failed */
  KC_EHIP = -3,          /* a HIP runtime call failed */
  KC_ERANK = -4,         /* least-squares design matrix rank-deficient or n_t < P */
  KC_ENOCONV = -5,       /* an iterative solve hit its iteration cap */
  KC_ENONFINITE = -6,    /* NaN or Inf met in a sample */
  KC_EUNSUPPORTED = -7   /* parameter combination not implemented */
};

enum { KC_PREC_F64 = 0, KC_PREC_F32_REFINED = 1 };
enum { KC_KLE_FIELD_EXP = 0, KC_KLE_SNAPSHOT = 1 };
/* initial guess of parareal_solve (Algorithm 3 step 6 and the comparators of Section 5) */
enum { KC_INIT_GIVEN = 0, KC_INIT_ZERO = 1, KC_INIT_COARSE = 2, KC_INIT_GPC = 3, KC_INIT_RANDOM = 4,
       KC_INIT_MLP = 5, KC_INIT_MLP_GPC_FALLBACK = 6 };
/* per-sample status written by parareal_solve */
enum { KC_SAMPLE_CONVERGED = 0, KC_SAMPLE_MAXITER = 1, KC_SAMPLE_NONFINITE = 2 };

typedef struct klecgc_ctx klecgc_ctx;
typedef struct klecgc_kle klecgc_kle;
typedef struct klecgc_gpc klecgc_gpc;
typedef struct klecgc_mlp klecgc_mlp;

/* One problem family (uniform batch).  Section 3.1: N coarse slices of length
 * dT = T/N, J fine steps of dt = dT/J per slice, backward Euler for F and G;
 * Section 3.2: alpha in (0,1) couples u(0) = alpha u(T) in the coarse model. */
typedef struct {
  int32_t dim;            /* 1 or 2 */
  int32_t n;              /* interior nodes per dimension (Nx = n^dim), n >= 1 */
  double  T;              /* horizon, > 0 */
  int32_t N;              /* coarse slices, power of two, 2 <= N <= 256 */
  int32_t J;              /* fine steps per slice, >= 1 */
  double  alpha;          /* twist parameter, 0 < alpha < 1 */
  double  forcing;        /* constant source f */
  int32_t precision;      /* KC_PREC_F64 or KC_PREC_F32_REFINED (2D fine path only) */
  double  tol;            /* parareal stop: max|U^{k+1}-U^k| / max|U^{k+1}| <= tol (> 0) */
  int32_t max_iter;       /* parareal iteration cap, >= 1 */
  double  inner_rtol;     /* 2D fine solves: FP64 residual <= inner_rtol * (|w|_inf + dt|f|)
                             + 8 eps max_p(diag_p) |w|_inf (the FP64 rounding floor of the
                             residual itself); 0 selects 1e-13 */
  int32_t inner_max_iter; /* 2D fine solves: Krylov iteration cap per solve; 0 selects 4000 */
  double  cgc_rtol;       /* 2D shifted solves of step (b): relative residual; 0 selects 1e-13
                             in cgc_diag_solve and 1e-7 inside parareal_solve (which solves
                             for the correction, see parareal_solve) */
  int32_t cgc_max_iter;   /* 2D shifted solves: iteration cap; 0 selects 20000 */
} klecgc_problem;

/* KL descriptor.
 * FIELD_EXP (input field; Section 2, separated representation): Gaussian field
 *   with covariance sigma^2 exp(-|x-y|/corr_len) on [0,1] (separable product in
 *   2D), closed-form eigenpairs, the d largest modes evaluated at the faces.
 * SNAPSHOT (solution snapshots; Section 2.1, Algorithm 3 steps 1-2, 4): rows of
 *   S are n_t flattened states of length L = N*Nx; modes kept by the smallest
 *   M_Q with eigenvalue fraction >= 1 - eps_kl, capped at numerical rank. */
typedef struct {
  int32_t kind;           /* KC_KLE_FIELD_EXP or KC_KLE_SNAPSHOT */
  int32_t dim, n, d;      /* FIELD_EXP */
  double  corr_len, sigma;/* FIELD_EXP */
  int64_t L;              /* SNAPSHOT: row length */
  double  eps_kl;         /* SNAPSHOT: truncation tolerance (e.g. 1e-10) */
} klecgc_kle_desc;

/* ---- lifecycle ---------------------------------------------------------- */
/* Create a context on `device` that enqueues on `hip_stream` (a hipStream_t;
 * NULL = the null stream).  The stream is borrowed, not owned. */
int klecgc_create(klecgc_ctx** out, int device, void* hip_stream);
void klecgc_destroy(klecgc_ctx* ctx);
int klecgc_set_stream(klecgc_ctx* ctx, void* hip_stream);
const char* klecgc_last_error(const klecgc_ctx* ctx);
void klecgc_kle_free(klecgc_kle* h);
void klecgc_gpc_free(klecgc_gpc* h);
void klecgc_mlp_free(klecgc_mlp* h);
/* Counters of the last call on ctx (instrumentation), out16[16]: [0..3] fine implicit
 * solves: total Krylov iterations, total float64 refinement passes, number of implicit
 * steps, max iterations of one solve; [4..7] the same for the shifted solves of step (b)
 * (2D only; passes unused); [8] shader-clock cycles of the 2D resident fine kernel summed
 * over work-groups, [9] of which inside its float32 Krylov loops; [10] fine implicit steps
 * and [11] shifted solves that ended above their residual target; [12..15] reserved (0).
 * After a model_* call on a nonlinear model: [0] Newton steps of all backward-Euler steps
 * (summed over systems), [2] those backward-Euler steps, [4] Newton steps of the coarse grid
 * corrections summed over samples, [7] the most one correction of one sample took, [10] the
 * backward-Euler steps whose Newton iteration reached newton_max_iter. */
int klecgc_last_stats(const klecgc_ctx* ctx, int64_t* out16);
/* Device time of the last call on ctx, measured with HIP events on the context stream
 * around each kernel launch (instrumentation): ms8[c] milliseconds and count8[c] launches
 * (count8 nullable) for the kernel classes c = 0 fine propagator, 1 shifted solves of
 * step (b), 2 forward slice FFT, 3 inverse slice FFT, 4 defect stencil, 5 prediction GEMM,
 * 6 MLP forward/backward/Adam. */
int klecgc_last_times(const klecgc_ctx* ctx, double* ms8, int64_t* count8);
/* Kernel choices for 2D KC_PREC_F32_REFINED problems of one grid size n, and the
 * float32 residual reduction each refinement pass asks of the inner Krylov loop (the
 * float64 residual targets inner_rtol / cgc_rtol are unaffected: they alone decide
 * when a solve stops).  Variants (-1 = built-in choice by n):
 *   fine:  KC_FINE_STREAM64 float64 PCG streaming through device memory (any n);
 *          KC_FINE_RES16/32/64/128 work-group-resident float32 PCG for n <= 16/32/64/128;
 *          KC_FINE_RB128 work-group-resident float32 CG on the red-black reduced system
 *          (odd-coloured nodes eliminated) for n <= 128;
 *          KC_FINE_MG float32 CG preconditioned by an aggregation-multigrid V-cycle,
 *          streaming through device memory (any n);
 *   shifted solves of step (b): KC_CGC_STREAM64 float64 COCG (any n);
 *          KC_CGC_RES16/32/64 work-group-resident float32 COCG for n <= 16/32/64;
 *          KC_CGC_STREAM32 float32 COCG streaming through device memory (any n);
 *          KC_CGC_MG32 float32 COCG preconditioned by an aggregation-multigrid V-cycle,
 *          streaming through device memory (any n). */
enum { KC_FINE_STREAM64 = 0, KC_FINE_RES16 = 1, KC_FINE_RES32 = 2, KC_FINE_RES64 = 3, KC_FINE_RES128 = 4,
       KC_FINE_MG = 5, KC_FINE_RB128 = 6 };
enum { KC_CGC_STREAM64 = 0, KC_CGC_RES16 = 1, KC_CGC_RES32 = 2, KC_CGC_RES64 = 3, KC_CGC_STREAM32 = 4,
       KC_CGC_MG32 = 5 };
typedef struct {
  int32_t fine_variant;    /* -1 or KC_FINE_* */
  float   fine_pcg_rtol;   /* in (0, 0.5); default 1e-6 */
  int32_t cgc_variant;     /* -1 or KC_CGC_* */
  float   cgc_inner_rtol;  /* in (0, 0.5); default 1e-5 */
  int32_t mg_sweeps;       /* smoothing sweeps per level and direction of the multigrid
                              variants, 1..4; 0 selects 2 */
  int32_t mg_smoother;     /* multigrid smoother: 0 red-black Gauss-Seidel, 1 damped Jacobi */
} klecgc_tuning;
/* Set / read the tuning the context uses for grid size n (KC_EINVAL if a variant does
 * not fit n or a tolerance or sweep count is out of range).  klecgc_get_tuning returns
 * the defaults (-1, 1e-6, -1, 1e-5, 0, 0) for an n never tuned. */
int klecgc_set_tuning(klecgc_ctx* ctx, int32_t n, const klecgc_tuning* t);
int klecgc_get_tuning(const klecgc_ctx* ctx, int32_t n, klecgc_tuning* t);
/* Autotuner: times every fitting fine variant (KC_FINE_MG only above n = 128, where no
 * resident variant fits) x per-pass reduction {1e-5, 3e-6, 1e-6,
 * 3e-7} (the faster of two timings each) on the first min(M, 16) samples of a_dev (fine
 * sweep over all N slices from the
 * coarse-propagator states), then every fitting shifted-solve variant x {1e-4, 3e-5,
 * 1e-5, 3e-6} (x multigrid smoothing {Gauss-Seidel 2, Gauss-Seidel 1, Jacobi 2} for
 * KC_CGC_MG32; a variant whose first timing is more than twice the best so far is not
 * timed further) on the defect those states
 * leave (correction tolerance cgc_rtol, default 1e-7), keeps the fastest of each for
 * prob->n in the context and returns it in *out
 * (nullable).  ms_out[2] (nullable): the winning fine and shifted-solve times.
 * prob must be 2D and KC_PREC_F32_REFINED (else KC_EUNSUPPORTED). */
int klecgc_autotune(klecgc_ctx* ctx, const klecgc_problem* prob, const double* a_dev, int64_t M,
                    klecgc_tuning* out, double* ms_out);
/* Library version string (static storage). */
const char* klecgc_version(void);

/* ---- KL ----------------------------------------------------------------- */
/* kle_build: FIELD_EXP ignores S_dev/n_t; SNAPSHOT reads S_dev [n_t][L] float64
 * (Section 2.1: mean, centred Gram matrix C = S~ S~^T / n_t on the device, its
 * eigenpairs on the host, basis g_k = (lam_k n_t)^{-1/2} S~^T e_k on the device).
 * *n_modes receives d (FIELD_EXP) or M_Q (SNAPSHOT). */
int kle_build(klecgc_ctx* ctx, const klecgc_kle_desc* desc, const double* S_dev, int64_t n_t,
              klecgc_kle** out, int32_t* n_modes);
/* kle_synthesize: a[m][f] = exp(sum_k sqrt(lam_k) phi_k(face f) xi[m][k]) for a
 * FIELD_EXP handle.  xi_dev [M][d] float64, a_dev [M][Fc] float64; a32_dev [M][Fc]
 * float32 (nullable) receives the same values rounded to nearest float32. */
int kle_synthesize(klecgc_ctx* ctx, const klecgc_kle* field, const double* xi_dev, int64_t M,
                   double* a_dev, float* a32_dev);
/* Copy a SNAPSHOT handle's mean [L] and scaled basis W = diag(sqrt(lam)) G
 * [M_Q][L] (row k = sqrt(lam_k) g_k) and eigenvalues [M_Q] to caller device memory
 * (any pointer may be NULL). */
int kle_export(klecgc_ctx* ctx, const klecgc_kle* snap, double* mean_dev, double* W_dev,
               double* lam_dev);

/* ---- gPC (Section 2.2; Algorithm 3 steps 3, 5, 6) ------------------------- */
/* univariate families of the Wiener-Askey table (Section 2.2): Gaussian inputs ~ N(0,1) take
 * orthonormal probabilists' Hermite polynomials, uniform inputs on [-1, 1] orthonormal
 * Legendre polynomials sqrt(2m+1) P_m (inputs uniform on [lo, hi] are mapped to [-1, 1] by
 * the caller) */
enum { KC_GPC_HERMITE = 0, KC_GPC_LEGENDRE = 1 };
/* gpc_fit: orthonormal tensor basis of the family `basis` of total degree <= p
 * in d variables (P = C(p+d, p) terms, degree-graded lexicographic order),
 * B[j][i] = psi_i(xi_j), D = zeta(xi_j) of the training snapshots of `snap`,
 * h = argmin |B h - D|_2 by Householder QR on the host.  xi_train_dev [n_t][d]
 * float64 must be the parameters of the rows of S given to kle_build.
 * Returns KC_ERANK if n_t < P or B is rank-deficient.  *P receives P. */
int gpc_fit(klecgc_ctx* ctx, const klecgc_kle* snap, const double* xi_train_dev, int64_t n_t,
            int32_t d, int32_t p, int32_t basis, klecgc_gpc** out, int32_t* P);
/* gpc_predict: U0[m] = u_bar + sum_i sqrt(lam_i) (sum_j h_{j,i} psi_j(xi_m)) g_i
 * (Algorithm 3 step 6).  xi_dev [M][d], U0_dev [M][L] float64. */
int gpc_predict(klecgc_ctx* ctx, const klecgc_gpc* gpc, const double* xi_dev, int64_t M,
                double* U0_dev);

/* ---- parareal building blocks ------------------------------------------- */
/* fine_propagate (Algorithm 2 step 1, eq. PGC_step1): for every sample m and
 * slice s, J backward-Euler steps of size dt = T/(N J) from start[m][s]:
 *     (I + dt A_m) w_{j+1} = w_j + dt f,   end[m][s] = w_J.
 * a_dev [M][Fc], start_dev and end_dev [M][N][Nx] float64 (may not alias).
 * active_dev [M] (nullable = all samples): samples with active_dev[m] == 0 are skipped
 * and their rows of end_dev are left untouched.
 * 1D: direct tridiagonal (Thomas) solves in float64.
 * 2D: precision F64 -> float64 Jacobi-PCG to inner_rtol; F32_REFINED ->
 * float32 Krylov corrections with float64 residuals and coefficients
 * until the float64 residual meets inner_rtol.  Returns KC_ENOCONV if a
 * solve hits inner_max_iter (results are still written). */
int fine_propagate(klecgc_ctx* ctx, const klecgc_problem* prob, const double* a_dev,
                   const double* start_dev, int64_t M, double* end_dev, const uint8_t* active_dev);
/* fine_propagate_noalloc: fine_propagate (same arguments, kernels and results) for callers
 * that cannot allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  It allocates nothing: its workspace (solver tables,
 * per-system increments, multigrid levels and Krylov vectors, the status block) comes from
 * a 64 MiB device array that the library holds on each GPU until the process ends.
 * Returns KC_EINVAL, before any output is written, if the call needs more than that
 * (roughly: 2D n <= 128 float32-refined needs 16 N Nx M bytes of increments plus 12 Nx M +
 * 8 n (n+1) M; 1D 24 n M; float64 PCG 24 N Nx M; n > 128 runs its multigrid systems in
 * chunks of what fits).  All calls on one GPU share the array: calls that overlap on one
 * GPU (several host threads or streams) race. */
int fine_propagate_noalloc(klecgc_ctx* ctx, const klecgc_problem* prob, const double* a_dev,
                           const double* start_dev, int64_t M, double* end_dev,
                           const uint8_t* active_dev);
/* cgc_diag_solve (Section 3.2, eq. matrix_NT and eq. three-steps): solves
 *     (C_alpha (x) I + dT I (x) A_m) u_m = r_m   for every sample m,
 * C_alpha the alpha-circulant time matrix, by (a) p = F_N^* Lambda r (real FFT
 * over slices, float64), (b) (lambda_k I + dT A) q_k = p_k for k = 0..N/2
 * (conjugate symmetry; complex Thomas in 1D, Jacobi-COCG in complex128 in 2D),
 * (c) u = Lambda^{-1} F_N q (float64).  Lambda = diag(alpha^{s/N}).
 * r_dev, u_dev [M][N][Nx] float64 (may alias). */
int cgc_diag_solve(klecgc_ctx* ctx, const klecgc_problem* prob, const double* a_dev,
                   const double* r_dev, int64_t M, double* u_dev);
/* coarse_propagate (Section 3.1, G): U[m][s] = G(U[m][s-1]) sequentially over
 * slices from u0 (NULL = 0): one backward-Euler step of dT per slice. */
int coarse_propagate(klecgc_ctx* ctx, const klecgc_problem* prob, const double* a_dev,
                     const double* u0_dev, int64_t M, double* U_dev);

/* serial_fine_propagate (the reference solution of Section 2 and Section 5):
 * U[m][s] = F(U[m][s-1]) sequentially over the slices from u0 (NULL = 0), F as in
 * fine_propagate.  The batched serial sweep, used as the accuracy reference and as
 * the time-serial baseline. */
int serial_fine_propagate(klecgc_ctx* ctx, const klecgc_problem* prob, const double* a_dev,
                          const double* u0_dev, int64_t M, double* U_dev);

/* ---- driver (Algorithms 2 and 3) ----------------------------------------- */
/* parareal_solve: parareal with diagonalised CGC for M samples.
 *   u0_dev [M][Nx] or NULL (zero initial condition);
 *   init (the initial guess U^0 [M][N][Nx]):
 *     KC_INIT_GIVEN   init_dev [M][N][Nx];
 *     KC_INIT_ZERO    U^0 = 0;
 *     KC_INIT_COARSE  one sequential G sweep from u0 (Section 3.1);
 *     KC_INIT_GPC     the gPC surrogate at xi_dev [M][d] (Algorithm 3 step 6; gpc required);
 *     KC_INIT_RANDOM  the random guess of the comparators of Section 5: entry i of U^0
 *                     (row-major over [M][N][Nx]) is the SplitMix64 output (Steele, Lea
 *                     and Flood, OOPSLA 2014) of the state seed + (i+1) 0x9E3779B97F4A7C15
 *                     (mod 2^64), its top 53 bits times 2^-53, i.i.d. U(0,1);
 *     KC_INIT_MLP     the learned guess of mlp_initial_guess at xi_dev [M][n_in] (mlp
 *                     required; its n_out must be N nc^2, nc the restricted grid);
 *     KC_INIT_MLP_GPC_FALLBACK  both the learned and the gPC guess (mlp, gpc, xi_dev
 *                     required); iteration 0's fine sweep runs on each, and a sample keeps
 *                     the gPC guess when its continuity defect
 *                         max_s |F(U^0_{s-1}) - U^0_s|_inf / max_s |U^0_s|_inf  (U^0_{-1} = u0)
 *                     is strictly smaller than the learned guess's, or when the learned
 *                     one's is NaN and the gPC one's is not (one fine sweep more than
 *                     KC_INIT_MLP; the sweep of the kept guess is iteration 0's);
 *   seed: KC_INIT_RANDOM only;
 *   U_dev [M][N][Nx] receives U^k at each sample's stop;
 *   iters_host [M], status_host [M] (KC_SAMPLE_*) host arrays;
 *   delta_hist_host [M][max_iter] (nullable) receives the increments
 *   (unused entries set to 0);
 *   guess_host [M] (nullable) receives the guess each sample started from: init, or
 *   KC_INIT_GPC for a sample that KC_INIT_MLP_GPC_FALLBACK moved to the gPC guess.
 * Each iteration: fine sweep over all active (sample, slice) pairs (the first
 * slice's F(u0) is computed once), defect d_s = (I + dT A)(F_s - U_s), one
 * cgc_diag_solve, U += correction; a sample stops when its increment
 * max|U^{k+1}-U^k| / max|U^{k+1}| <= tol.  In exact arithmetic the iterates
 * equal those of Algorithm 2 (the correction form solves the same
 * all-at-once system for U^{k+1} - U^k). */
int parareal_solve(klecgc_ctx* ctx, const klecgc_problem* prob, const double* a_dev,
                   const double* u0_dev, int64_t M, int32_t init, const double* init_dev,
                   const klecgc_gpc* gpc, klecgc_mlp* mlp, const double* xi_dev, uint64_t seed,
                   double* U_dev, int32_t* iters_host, int32_t* status_host,
                   double* delta_hist_host, int32_t* guess_host);

/* parareal_solve_sequential (Section 3.1, Algorithm 1, eq. pred_correc): parareal with the
 * sequential coarse grid correction, the comparator of Section 5 ("standard parareal"):
 *     U^{k+1}_1 = F(u0),  U^{k+1}_s = G(U^{k+1}_{s-1}) + F(U^k_{s-1}) - G(U^k_{s-1}),
 * G one backward-Euler step of dT = T/N.  The fine sweep and the coarse steps of the old
 * starts run over all slices at once; the correction sweeps the N slices in order (one
 * batched coarse step per slice).  alpha is not used.  Arguments as parareal_solve, with
 * init any mode but KC_INIT_MLP_GPC_FALLBACK (KC_EUNSUPPORTED); the stop rule is the same
 * increment test.  In exact arithmetic U^N is the serial fine solution (finite termination). */
int parareal_solve_sequential(klecgc_ctx* ctx, const klecgc_problem* prob, const double* a_dev,
                              const double* u0_dev, int64_t M, int32_t init, const double* init_dev,
                              const klecgc_gpc* gpc, klecgc_mlp* mlp, const double* xi_dev, uint64_t seed,
                              double* U_dev, int32_t* iters_host, int32_t* status_host,
                              double* delta_hist_host);

/* ---- ragged batches ------------------------------------------------------------
 * Samples of one problem family that differ in grid size n and slice count N, solved
 * together by the iteration of parareal_solve (Algorithm 2 with the diagonalised CGC of
 * Section 3.2).  Sample m has n = tasks[m].n and N = tasks[m].N; its faces a [Fc(n)]
 * start at element tasks[m].face_off of a_dev, its states U [N][n^dim] at element
 * tasks[m].state_off of U_dev (float64).  Regions of different samples must not
 * overlap.  The other parameters come from *base (its n and N are ignored); u0 = 0.
 * Samples of equal (n, N) form a class; classes run concurrently, each on its own
 * stream.  With KC_BATCH_GRAPH, the first iteration runs eagerly and one iteration of
 * all classes is then captured into a HIP graph and replayed until every sample has
 * stopped (convergence is tested on the device).
 *   init: KC_INIT_ZERO, KC_INIT_COARSE, or KC_INIT_GIVEN (U_dev holds the guess);
 *   iters_host [M], status_host [M] (KC_SAMPLE_*) as in parareal_solve;
 *   latency_ms_host [M] (nullable): time from the start of the call to the iteration
 *   at which the sample stopped (device clock); total_ms_host (nullable): wall time of
 *   the call on the context stream.
 * With KC_BATCH_GRAPH the call must not be made while the context stream is being
 * captured by the caller (it captures on a library-owned stream of its own). */
typedef struct {
  int32_t n;          /* interior nodes per dimension */
  int32_t N;          /* coarse slices (power of two, 2..256) */
  int64_t face_off;   /* element offset of the sample's faces in a_dev */
  int64_t state_off;  /* element offset of the sample's N * n^dim states in U_dev */
} klecgc_task;
/* flags: KC_BATCH_GRAPH as above; KC_BATCH_PROGRESS prints one line per iteration to stderr
 * (iteration index, samples still active, elapsed seconds) so a long call is never silent;
 * KC_BATCH_PERSISTENT runs the classes from one host thread, and the fine sweeps of all
 * classes with n <= 128 (2D, KC_PREC_F32_REFINED) of an iteration as ONE persistent launch:
 * its work-groups take (class, sample, slice) tasks from device counters (eight ranges, one
 * per XCD, then from each other's) and skip the samples already retired; each task is solved
 * by the red-black resident kernel (so a class gives the results of the uniform driver with
 * fine variant KC_FINE_RB128, bit for bit), and the iterations after the first are replayed
 * from one graph holding that launch and every class's correction branch.  Other classes
 * run their own fine sweeps in their branches. */
enum { KC_BATCH_GRAPH = 1, KC_BATCH_PROGRESS = 2, KC_BATCH_PERSISTENT = 4 };
int parareal_solve_batch(klecgc_ctx* ctx, const klecgc_problem* base, const klecgc_task* tasks,
                         int64_t M, const double* a_dev, int32_t init, double* U_dev, int32_t flags,
                         int32_t* iters_host, int32_t* status_host, double* latency_ms_host,
                         double* total_ms_host);

/* ---- the model problems of Section 5 ------------------------------------------------
 * Batches of one of the paper's example problems, each sample with its own scalar parameter
 * c_dev[m] (float64 [M]):
 *   KC_MODEL_ADE_P1 (Section 5.1): u_t - div(a grad u) + b . grad u = f on (0,1)^2, zero
 *     Dirichlet data, a = c[m] (the paper's 0.5 (2 + cos(pi xi)^2)), b = beta (x2, x1),
 *     f = exp(-t) (g0 + a g1) with g1 = pi^2 sin(pi x1) sin(2 pi x2),
 *     g0 = -sin(pi x1) sin(2 pi x2) + beta pi (x2 cos(pi x1) sin(2 pi x2) / 2 + x1 sin(pi x1)
 *     cos(2 pi x2)), u(0) = sin(pi x1) sin(2 pi x2).  P1 elements on the uniform grid of n x n
 *     interior nodes (h = 1/(n+1)), each cell cut by its diagonal from (x_i, y_j) to
 *     (x_{i+1}, y_{j+1}); mass, stiffness and advection integrated exactly; load = the
 *     consistent mass matrix times the nodal interpolant of f (boundary nodes included).
 *     Unknown of interior node (i, j) (0-based) is j*n + i.  One backward-Euler step of size
 *     tau ending at t: (M + tau (a K + B)) w' = M w + tau F(t).  n <= 31.
 *   KC_MODEL_BURGERS (Section 5.2): u_t + u u_x = (c[m]/50) u_xx on (0,1), u = 0 at both ends,
 *     n interior nodes (h = 1/(n+1)), central second differences, first-order upwinding of
 *     u u_x by the sign of u_i; u(0) = sin(pi x).
 *   KC_MODEL_ALLEN_CAHN (Section 5.3): u_t - c[m] u_xx + u^3 - u = 0 on (-1,1), u(-1) = -1,
 *     u(1) = 1, n interior nodes (h = 2/(n+1)), central differences; u(0) = 0.53 x +
 *     0.47 sin(-1.5 pi x).  2 <= n <= 512 for both nonlinear models.
 *   The nonlinear models take each backward-Euler step w - tau f(w) = v by Newton's method
 *   from w = v with the exact (tridiagonal) Jacobian until the newton_tol test holds or
 *   newton_max_iter steps have run (the last iterate is kept; klecgc_last_stats counts such
 *   steps); the linear systems are solved by parallel cyclic reduction.
 * States are [M][N][Nx] float64 (Nx = n^2 for the 2D model, n in 1D).  The coarse problem
 * of Algorithm 2 couples U_0 = alpha U_N; with the mass matrix its all-at-once system is
 * (C_alpha (x) M + dT I (x) L) u = r (Section 3.2 with M in front of the time derivative). */
enum { KC_MODEL_ADE_P1 = 1, KC_MODEL_BURGERS = 2, KC_MODEL_ALLEN_CAHN = 3 };
typedef struct {
  int32_t model;           /* KC_MODEL_* */
  int32_t n;               /* interior nodes per dimension */
  double  T;               /* horizon, > 0 */
  int32_t N;               /* coarse slices, 2 <= N <= 64 (any N: the slice transforms are dense) */
  int32_t J;               /* fine steps per slice, >= 1 */
  double  alpha;           /* twist parameter, 0 < alpha < 1 */
  double  tol;             /* parareal stop on the increment (as parareal_solve); 0 runs max_iter */
  int32_t max_iter;        /* iteration cap, 1 <= max_iter <= 1000 */
  double  beta;            /* KC_MODEL_ADE_P1: advection scale (b = beta (x2, x1)) */
  double  newton_tol;      /* nonlinear models: Newton stop, |increment|_inf <= newton_tol
                              max(|u|_inf, 1), for the backward-Euler steps and the coarse grid
                              correction alike; 0 selects 1e-13 */
  int32_t newton_max_iter; /* nonlinear models: Newton cap per solve; 0 selects 50 */
} klecgc_model;
/* model_fine_propagate: end[m][s] = F(start[m][s]) over slice s (J backward-Euler steps of
 * dt = T/(N J); for the advection-diffusion model with the time-dependent load of slice s).
 * start_dev, end_dev [M][N][Nx] (may not alias).  KC_ENONFINITE if a sample's step matrix has
 * a zero or non-finite pivot (advection-diffusion model). */
int model_fine_propagate(klecgc_ctx* ctx, const klecgc_model* mp, const double* c_dev,
                         const double* start_dev, int64_t M, double* end_dev);
/* model_coarse_propagate / model_serial_fine: U[m][s] = G(U[m][s-1]) (one step of dT) or
 * F(U[m][s-1]) sequentially from u0_dev [M][Nx] (NULL = the model's initial value). */
int model_coarse_propagate(klecgc_ctx* ctx, const klecgc_model* mp, const double* c_dev,
                           const double* u0_dev, int64_t M, double* U_dev);
int model_serial_fine(klecgc_ctx* ctx, const klecgc_model* mp, const double* c_dev,
                      const double* u0_dev, int64_t M, double* U_dev);
/* model_cgc_solve (Algorithm 2 step 2, Section 3.2): from the iterate Uk_dev and the fine
 * results F_dev (F_dev[m][0] = F(u0), F_dev[m][s] = F(Uk[m][s-1])), both [M][N][Nx], the new
 * iterate Unew_dev [M][N][Nx] (may alias Uk_dev).  The linear model solves the all-at-once
 * system once by the three steps of eq. three-steps (dense transforms over the N slices,
 * banded LU of the N/2+1 shifted systems (lambda_k M + dT L)); the nonlinear models run the
 * simplified Newton iteration of eq. Newton2 with the averaged Jacobian of eq. Jac, each
 * Newton step by the same three steps; newton_its_host [M] (nullable) receives its counts. */
int model_cgc_solve(klecgc_ctx* ctx, const klecgc_model* mp, const double* c_dev, const double* Uk_dev,
                    const double* F_dev, int64_t M, double* Unew_dev, int32_t* newton_its_host);
/* model_parareal_solve (Algorithms 2 and 3) and model_parareal_solve_sequential
 * (Algorithm 1): arguments as parareal_solve, with
 *   init KC_INIT_GIVEN | ZERO | COARSE | GPC | RANDOM (the gPC surrogate's L must be N Nx);
 *   u0_dev [M][Nx] or NULL (the model's initial value);
 *   ref_dev [M][N][Nx] (nullable): a reference solution (the serial fine solution of
 *   Section 5) for the error history err_hist_host [M][max_iter+1][N] (nullable; needs
 *   ref_dev): entry [m][k][s] = max_p |U^k[m][s][p] - ref[m][s][p]|, k = 0 the guess;
 *   rows after a sample's stop repeat its last iterate's errors.
 * With tol = 0 every sample runs exactly max_iter iterations (status KC_SAMPLE_MAXITER). */
int model_parareal_solve(klecgc_ctx* ctx, const klecgc_model* mp, const double* c_dev,
                         const double* u0_dev, int64_t M, int32_t init, const double* init_dev,
                         const klecgc_gpc* gpc, const double* xi_dev, uint64_t seed,
                         const double* ref_dev, double* U_dev, int32_t* iters_host, int32_t* status_host,
                         double* delta_hist_host, double* err_hist_host);
int model_parareal_solve_sequential(klecgc_ctx* ctx, const klecgc_model* mp, const double* c_dev,
                                    const double* u0_dev, int64_t M, int32_t init, const double* init_dev,
                                    const klecgc_gpc* gpc, const double* xi_dev, uint64_t seed,
                                    const double* ref_dev, double* U_dev, int32_t* iters_host,
                                    int32_t* status_host, double* delta_hist_host, double* err_hist_host);

/* ---- learned initial guess (replaces the gPC map of Algorithm 3 step 6) ------
 * A multilayer perceptron maps xi [d] to the states of all N slices restricted to an
 * nc x nc grid (n_out = N nc^2), trained on solutions the method produced:
 *     pre1 = X W1 + b1, h1 = GELU(pre1); pre2 = h1 W2 + b2, h2 = GELU(pre2);
 *     Y = h2 W3 + b3;  loss = mean((Y - T)^2) on per-output z-scored targets.
 * GELU is x Phi(x) (exact erf).  GEMMs run on BF16 MFMA with FP32 accumulation;
 * the operands X, W1..W3, h1, h2 and the backward products dY, dpre2, dpre1 are
 * rounded to bfloat16 (nearest even).  Adam (beta1 0.9, beta2 0.999, eps 1e-8,
 * bias-corrected) updates FP32 master weights.
 * Flat parameter layout (FP32): W1 [n_in][H], b1 [H], W2 [H][H], b2 [H],
 * W3 [H][n_out], b3 [n_out]; n_params = n_in H + H + H H + H + H n_out + n_out.
 * Grid transfer (2D): bilinear interpolation with zero boundary values between the
 * n x n grid (h = 1/(n+1)) and the nc x nc grid (H = 1/(nc+1)), evaluated at the
 * nodes of the target grid; both x fastest. */
/* Allocate a network (weights zero, normalisation identity).  1 <= n_in <= 4096,
 * 1 <= hidden <= 16384, hidden * n_out < 2^31.  *n_params (nullable) receives the
 * flat parameter count. */
int mlp_create(klecgc_ctx* ctx, int32_t n_in, int32_t hidden, int64_t n_out, klecgc_mlp** out,
               int64_t* n_params);
/* Load FP32 parameters params_dev [n_params] (e.g. a seeded initialisation drawn by
 * the caller) and reset the Adam state. */
int mlp_set_params(klecgc_ctx* ctx, klecgc_mlp* h, const float* params_dev);
/* Copy the FP32 parameters [n_params] and the target mean / std [n_out] to device
 * memory (each pointer nullable). */
int mlp_get_params(klecgc_ctx* ctx, const klecgc_mlp* h, float* params_dev, float* mean_dev,
                   float* std_dev);
/* Y_dev [n][n_out] FP32: store the per-output mean and population standard deviation
 * over the n rows in the handle (std 0 is replaced by 1) and z-score Y in place. */
int mlp_normalize_targets(klecgc_ctx* ctx, klecgc_mlp* h, float* Y_dev, int64_t n);
/* Adam training: `epochs` passes over the n rows, mini-batches of `batch` consecutive
 * rows of the order perm_dev [epochs][n] int32 (nullable = identity; each row a
 * permutation of 0..n-1), one Adam step per mini-batch.  Learning rate of epoch e:
 * lr (lr_final/lr)^(e/(epochs-1)) (geometric decay; lr_final <= 0 keeps lr).
 * KC_EINVAL if a perm entry lies outside [0, n).  One epoch is captured into a HIP graph on
 * a library-owned stream and replayed, so the call must not be made while the context
 * stream is being captured by the caller.
 * xi_dev [n][n_in] float64, Y_dev [n][n_out] z-scored FP32 targets.
 * loss_host [epochs] (nullable) receives the mean of the per-batch losses weighted by
 * batch size (evaluated before each step). */
int mlp_train(klecgc_ctx* ctx, klecgc_mlp* h, const double* xi_dev, const float* Y_dev, int64_t n,
              int32_t epochs, int32_t batch, float lr, float lr_final, const int32_t* perm_dev,
              float* loss_host);
/* Y_dev [M][n_out] FP32 = network output (normalised units) for xi_dev [M][n_in]. */
int mlp_predict(klecgc_ctx* ctx, klecgc_mlp* h, const double* xi_dev, int64_t M, float* Y_dev);
/* Gradient of the loss of one batch (all n rows, n <= 65535) at the current
 * parameters into grads_dev [n_params] FP32 (flat layout); *loss_host (nullable)
 * receives the loss.  Parameters and Adam state are unchanged. */
int mlp_grad(klecgc_ctx* ctx, klecgc_mlp* h, const double* xi_dev, const float* Y_dev, int64_t n,
             float* grads_dev, double* loss_host);
/* Restriction: Yc[r] = the bilinear interpolant of U[r] (n x n) at the nc x nc nodes,
 * for r < R.  U_dev [R][n*n] float64, Yc_dev [R][nc*nc] FP32. */
int grid_restrict(klecgc_ctx* ctx, int32_t n, int32_t nc, const double* U_dev, int64_t R,
                  float* Yc_dev);
/* Learned initial guess for parareal_solve (KC_INIT_GIVEN): U0[m][s] = bilinear
 * prolongation to n x n of mean + std * Y[m][s] (Y = mlp_predict(xi)[m] read as
 * [N][nc*nc]).  Requires n_out = N nc^2.  xi_dev [M][n_in], U0_dev [M][N][n*n]. */
int mlp_initial_guess(klecgc_ctx* ctx, klecgc_mlp* h, int32_t n, int32_t nc, int32_t N,
                      const double* xi_dev, int64_t M, double* U0_dev);

#ifdef __cplusplus
}
#endif
#endif /* KLECGC_H */
