// Internal declarations of the Section 5 model problems (the model_* entry points): the P1
// finite-element advection-diffusion problem (ade.hip), Burgers and Allen-Cahn (nonlinear.hip),
// and the slice transforms of any length N they share (spectral.hip).
#pragma once

#include "common.h"

namespace kc {

// complex float64 as a plain pair (device and host)
struct cplx {
  double re, im;
};

// Validates a model descriptor (throws KC_EINVAL / KC_EUNSUPPORTED).
void validate_model(const klecgc_model& mp);
inline int64_t model_nx(const klecgc_model& mp) {
  return mp.model == KC_MODEL_ADE_P1 ? (int64_t)mp.n * mp.n : (int64_t)mp.n;
}
// number of distinct shifted systems per sample in step (b) (conjugate symmetry)
inline int model_bins(int N) { return N / 2 + 1; }

// ---- slice transforms of eq. three-steps for any N (spectral.hip) ---------------------
// Per-call tables: twiddles w_m = (cos 2 pi m / N, sin 2 pi m / N), m < N, and the scaling
// Lambda_s = alpha^{s/N}, s < N, written to the 3 N doubles at d (device memory).
struct SliceTables {
  const double* tw;    // [N][2]
  const double* lam;   // [N]
};
SliceTables slice_tables(klecgc_ctx* ctx, int N, double alpha, double* d);
// spec[m][k][p] = N^{-1/2} sum_s conj(w^{ks}) Lambda_s D[m][s][p], k < N/2+1, for the listed
// samples (list nullable = 0..nlist-1); spec is [M][N/2+1][Nx] complex.
void launch_slice_dft(hipStream_t st, const double* D, const int32_t* list, int64_t nlist, int N, int64_t Nx,
                      const SliceTables& tb, cplx* spec);
// U[m][s][p] (+)= Lambda_s^{-1} N^{-1/2} sum_{k<N} w^{ks} q_k (real part; q_{N-k} = conj q_k);
// maxima[2m] = max |increment|, maxima[2m+1] = max |U| after the update (as ordered bit
// patterns of non-negative doubles; NaN wins), for the listed samples.
void launch_slice_idft(hipStream_t st, const cplx* spec, const int32_t* list, int64_t nlist, int N, int64_t Nx,
                       const SliceTables& tb, double* U, bool accumulate, unsigned long long* maxima);
// err[m][s] = max_p |U[m][s][p] - ref[m][s][p]| (atomic max into err zeroed by the caller)
void launch_slice_error(hipStream_t st, const double* U, const double* ref, const int32_t* list, int64_t nlist,
                        int N, int64_t Nx, unsigned long long* err);

// SplitMix64 random guess (batch.hip): U[i] = top 53 bits of SplitMix64(seed + (i+1) golden) * 2^-53
void launch_random_guess(hipStream_t st, uint64_t seed, int64_t n, double* U);

// ---- drivers ---------------------------------------------------------------------
// model_* entry points (the argument checks are done by the caller)
int model_fine_impl(klecgc_ctx* ctx, const klecgc_model& mp, const double* c, const double* start, int64_t M,
                    double* end);
int model_coarse_impl(klecgc_ctx* ctx, const klecgc_model& mp, const double* c, const double* u0, int64_t M,
                      double* U);
int model_serial_fine_impl(klecgc_ctx* ctx, const klecgc_model& mp, const double* c, const double* u0, int64_t M,
                           double* U);
int model_cgc_impl(klecgc_ctx* ctx, const klecgc_model& mp, const double* c, const double* Uk, const double* Fv,
                   int64_t M, double* Unew, int32_t* newton_its);
struct ModelSolveArgs {
  const double* c;
  const double* u0;        // nullable: the model's own initial value
  int64_t M;
  GuessArgs guess;
  const double* ref;       // nullable: reference for the error history
  double* U;
  int32_t* iters;
  int32_t* status;
  double* delta_hist;      // [M][max_iter] nullable
  double* err_hist;        // [M][max_iter+1][N] nullable (needs ref)
  bool sequential;         // Algorithm 1 instead of Algorithms 2/3
};
int model_parareal_impl(klecgc_ctx* ctx, const klecgc_model& mp, const ModelSolveArgs& a);

// ---- the advection-diffusion model (ade.hip) -------------------------------------------
// F on slices [s_lo, s_lo + nsl) of the listed samples (J steps of tau = dT/J) or, with
// coarse, one step of dT; start of (m, s): shift ? (s == 0 ? u0[m] : base[m][s-1]) : base[m][s].
struct AdeSweep {
  const double* base;
  const double* u0;       // [M][Nx]
  bool shift;
  int s_lo, nsl;
  bool coarse;
  double* out;            // [M][N][Nx]
};
struct AdeState;   // per-call tables and factors
AdeState* ade_prepare(klecgc_ctx* ctx, const klecgc_model& mp, const double* c, int64_t M, bool need_coarse,
                      bool need_shifted);
void ade_release(AdeState* s);
void ade_sweep(klecgc_ctx* ctx, AdeState* s, const int32_t* list, int64_t nlist, const AdeSweep& sw);
void ade_initial_value(klecgc_ctx* ctx, const klecgc_model& mp, int64_t M, double* u0);
// CGC in correction form: U += solution of (C_alpha (x) M + dT I (x) L) dU = (M + dT L)(F - U)
void ade_correct(klecgc_ctx* ctx, AdeState* s, const int32_t* list, int64_t nlist, const double* Fv, double* U,
                 unsigned long long* maxima);
int ade_bad_samples(klecgc_ctx* ctx, AdeState* s, std::vector<uint8_t>& bad);

// ---- the nonlinear models (nonlinear.hip) -------------------------------------------------
struct NLState;   // per-call parameters, Newton bookkeeping and the correction's buffers
NLState* nl_prepare(klecgc_ctx* ctx, const klecgc_model& mp, const double* c, int64_t M, bool need_cgc);
void nl_release(NLState* s);
void nl_initial_value(klecgc_ctx* ctx, const klecgc_model& mp, int64_t M, double* u0);
// mode 0: start base[m][s]; 1: s == 0 ? u0[m] : base[m][s-1]; 2: s == 0 ? alpha base[m][N-1] : base[m][s-1]
void nl_sweep(klecgc_ctx* ctx, NLState* s, const int32_t* list, int64_t nlist, const double* base, const double* u0,
              int mode, int s_lo, int nsl, bool coarse, double* out);
// Newton coarse grid correction of the listed samples (list on the device and on the host;
// dev_newton_list: device scratch of M int32); maxima as ade_correct
void nl_correct(klecgc_ctx* ctx, NLState* s, const int32_t* list, const std::vector<int32_t>& hlist,
                int32_t* dev_newton_list, const double* Fv, double* U, unsigned long long* maxima);
int nl_failed_samples(klecgc_ctx* ctx, NLState* s, std::vector<uint8_t>& bad);
const std::vector<int64_t>& nl_newton_counts(const NLState* s);
// Newton steps, backward-Euler steps and steps whose Newton iteration reached its cap, of all
// sweeps since nl_prepare (summed over systems)
void nl_sweep_counts(klecgc_ctx* ctx, const NLState* s, int64_t* newton, int64_t* steps, int64_t* capped);
int64_t nl_newton_total(const NLState* s);
int nl_newton_max(const NLState* s);

}  // namespace kc
