// Autotuner for the 2D float32-refined path: for one grid size it times the kernel
// variants that fit (work-group-resident or streaming Krylov solvers) and the float32
// residual reduction asked of each refinement pass, on a small probe batch of the
// caller's samples, and keeps the fastest in the context's tuning table.  The float64
// residual targets, and so the results' accuracy, do not depend on these choices.
#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "common.h"

namespace kc {

namespace {
struct Buf {
  void* p = nullptr;
  explicit Buf(size_t bytes) {
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      throw Error{KC_ENOMEM, "autotuner buffer allocation failed"};
    }
  }
  ~Buf() {
    if (p) (void)hipFree(p);
  }
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
};
}  // namespace

int autotune_impl(klecgc_ctx* ctx, const klecgc_problem& p, const double* a, int64_t M, klecgc_tuning* out,
                  double* ms_out) {
  KC_REQUIRE(p.dim == 2 && p.precision == KC_PREC_F32_REFINED, KC_EUNSUPPORTED,
             "the autotuner serves 2D float32-refined problems");
  hipStream_t st = ctx->stream;
  const int n = p.n;
  // up to 16 samples: at 128^2 and 64 slices that is four rounds of work-groups over the
  // device, so a timing is not decided by the slowest single work-group
  const int64_t Mp = std::min<int64_t>(M, 16);
  const int64_t Nx = n_unknowns(p);
  const int64_t S = (int64_t)p.N * Nx;
  const int K = p.N / 2 + 1;
  Buf U(sizeof(double) * Mp * S), Fv(sizeof(double) * Mp * S), D(sizeof(double) * Mp * S);
  Buf spec0(sizeof(double) * 2 * Mp * K * Nx), spec(sizeof(double) * 2 * Mp * K * Nx);
  // probe states: one coarse sweep from zero (the states parareal starts from)
  coarse_sweep_impl(ctx, p, a, nullptr, Mp, (double*)U.p);
  const bool had = ctx->tuning.count(n) > 0;
  const KcTuning saved = tuning_for(ctx, n);
  KcTuning best = saved;
  double best_fine = std::numeric_limits<double>::infinity();
  double best_cgc = std::numeric_limits<double>::infinity();
  const float fine_rtols[] = {1e-5f, 3e-6f, 1e-6f, 3e-7f};
  const float cgc_rtols[] = {1e-4f, 3e-5f, 1e-5f, 3e-6f};
  auto restore = [&]() {   // on an error: the tuning the context had before
    if (had)
      ctx->tuning[n] = saved;
    else
      ctx->tuning.erase(n);
  };
  try {
    // ---- fine propagator
    for (int v : {KC_FINE_RES16, KC_FINE_RES32, KC_FINE_RES64, KC_FINE_RES128, KC_FINE_RB128, KC_FINE_MG}) {
      if (!fine_variant_fits(v, n)) continue;
      // up to 128^2 a system fits one CU and the resident kernels beat the streamed multigrid
      // path several times over (9x at 128^2, measured); it is timed only above
      if (v == KC_FINE_MG && n <= 128) continue;
      bool warmed = false;
      for (float r : fine_rtols) {
        KcTuning t = saved;
        t.fine_variant = v;
        t.fine_pcg_rtol = r;
        ctx->tuning[n] = t;
        FineArgs fa{a, (const double*)U.p, nullptr, true, 0, nullptr, (double*)Fv.p, Mp};
        if (!warmed) {
          (void)fine_propagate_impl(ctx, p, fa);
          warmed = true;
        }
        // the faster of two timings
        double ms = std::numeric_limits<double>::infinity();
        int rc = KC_OK;
        for (int rep = 0; rep < 2 && rc == KC_OK; ++rep) {
          const double t0 = ctx->ktime[KT_FINE];
          rc = fine_propagate_impl(ctx, p, fa);
          ms = std::min(ms, ctx->ktime[KT_FINE] - t0);
        }
        if (rc == KC_OK && ms < best_fine) {
          best_fine = ms;
          best.fine_variant = v;
          best.fine_pcg_rtol = r;
        }
        // a variant more than twice as slow as the best so far is not timed further
        if (rc == KC_OK && ms > 2.0 * best_fine) break;
      }
    }
    KC_REQUIRE(best_fine < std::numeric_limits<double>::infinity(), KC_ENOCONV,
               "no fine-propagator variant converged on the probe batch");
    // ---- shifted solves of step (b), on the defect the probe states leave
    ctx->tuning[n] = best;
    FineArgs fa{a, (const double*)U.p, nullptr, true, 0, nullptr, (double*)Fv.p, Mp};
    (void)fine_propagate_impl(ctx, p, fa);
    launch_defect(st, p, a, (const double*)Fv.p, (const double*)U.p, nullptr, Mp, (double*)D.p);
    launch_fft_forward(st, p, (const double*)D.p, nullptr, Mp, (double*)spec0.p);
    klecgc_problem pb = p;
    if (pb.cgc_rtol <= 0) pb.cgc_rtol = 1e-7;
    for (int v : {KC_CGC_RES16, KC_CGC_RES32, KC_CGC_RES64, KC_CGC_STREAM32, KC_CGC_MG32}) {
      if (!cgc_variant_fits(v, n)) continue;
      bool warmed = false;
      // multigrid smoothing (sweeps, smoother): Gauss-Seidel 2 and 1, Jacobi 2
      const int smoothing[3][2] = {{2, 0}, {1, 0}, {2, 1}};
      for (const auto& sm : smoothing)
      for (float r : cgc_rtols) {
        // only the multigrid variant smooths
        if (v != KC_CGC_MG32 && (sm[0] != 2 || sm[1] != 0)) continue;
        KcTuning t = best;
        t.cgc_variant = v;
        t.cgc_inner_rtol = r;
        t.mg_sweeps = v == KC_CGC_MG32 ? sm[0] : best.mg_sweeps;
        t.mg_smoother = v == KC_CGC_MG32 ? sm[1] : best.mg_smoother;
        ctx->tuning[n] = t;
        if (!warmed) {
          KC_TRY_HIP(hipMemcpyAsync(spec.p, spec0.p, sizeof(double) * 2 * Mp * K * Nx, hipMemcpyDeviceToDevice, st));
          (void)shifted_solve_impl(ctx, pb, a, nullptr, Mp, (double*)spec.p);
          warmed = true;
        }
        double ms = std::numeric_limits<double>::infinity();
        int rc = KC_OK;
        for (int rep = 0; rep < 2 && rc == KC_OK; ++rep) {   // the faster of two timings
          KC_TRY_HIP(hipMemcpyAsync(spec.p, spec0.p, sizeof(double) * 2 * Mp * K * Nx, hipMemcpyDeviceToDevice, st));
          const double t0 = ctx->ktime[KT_SHIFTED];
          rc = shifted_solve_impl(ctx, pb, a, nullptr, Mp, (double*)spec.p);
          ms = std::min(ms, ctx->ktime[KT_SHIFTED] - t0);
        }
        if (rc == KC_OK && ms < best_cgc) {
          best_cgc = ms;
          best.cgc_variant = v;
          best.cgc_inner_rtol = r;
          best.mg_sweeps = t.mg_sweeps;
          best.mg_smoother = t.mg_smoother;
        }
        if (rc == KC_OK && ms > 2.0 * best_cgc) break;   // as for the fine variants
      }
    }
  } catch (...) {
    restore();
    throw;
  }
  KC_TRY_HIP(hipStreamSynchronize(st));
  ctx->tuning[n] = best;
  if (out) {
    out->fine_variant = best.fine_variant;
    out->fine_pcg_rtol = best.fine_pcg_rtol;
    out->cgc_variant = best.cgc_variant;
    out->cgc_inner_rtol = best.cgc_inner_rtol;
    out->mg_sweeps = best.mg_sweeps;
    out->mg_smoother = best.mg_smoother;
  }
  if (ms_out) {
    ms_out[0] = best_fine;
    ms_out[1] = best_cgc;
  }
  return KC_OK;
}

}  // namespace kc
