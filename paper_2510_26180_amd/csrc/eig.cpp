// Eigen-decomposition of the snapshot Gram matrix (Section 2.1; Algorithm 3 step 2) on
// the device.  The n_t x n_t matrix is dense and symmetric; rocSOLVER's divide-and-conquer
// solver (syevd) runs it on the GPU, which keeps the offline stage practical at
// n_t in the thousands.  It is not on the per-solve path.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <vector>

#include "common.h"

namespace kc {

namespace {
rocblas_handle blas_handle(klecgc_ctx* ctx) {
  if (!ctx->blas) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) throw Error{KC_EHIP, "rocblas_create_handle failed"};
    ctx->blas = h;
  }
  rocblas_handle h = (rocblas_handle)ctx->blas;
  if (rocblas_set_stream(h, ctx->stream) != rocblas_status_success) throw Error{KC_EHIP, "rocblas_set_stream failed"};
  return h;
}
}  // namespace

void release_blas(klecgc_ctx* ctx) {
  if (ctx->blas) {
    (void)rocblas_destroy_handle((rocblas_handle)ctx->blas);
    ctx->blas = nullptr;
  }
}

// Cd: device n x n symmetric (only the upper triangle of its column-major reading is
// referenced; it is overwritten).  On return V (host, row-major n x n) holds the
// eigenvectors as columns and w the eigenvalues, both in descending eigenvalue order.
void gram_eig(klecgc_ctx* ctx, int n, double* Cd, std::vector<double>& V, std::vector<double>& w) {
  hipStream_t s = ctx->stream;
  rocblas_handle h = blas_handle(ctx);
  double* D = (double*)ctx->ws.get(WS_GEMM_A, sizeof(double) * 2 * (size_t)n + 256);
  double* E = D + n;
  int* info = (int*)(E + n);
  rocblas_status st = rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, n, Cd, n, D, E, info);
  if (st != rocblas_status_success) throw Error{KC_EHIP, "rocsolver_dsyevd failed (status " + std::to_string((int)st) + ")"};
  std::vector<double> cm((size_t)n * n), d(n);
  int hinfo = 0;
  KC_TRY_HIP(hipMemcpyAsync(cm.data(), Cd, sizeof(double) * cm.size(), hipMemcpyDeviceToHost, s));
  KC_TRY_HIP(hipMemcpyAsync(d.data(), D, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  KC_TRY_HIP(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, s));
  KC_TRY_HIP(hipStreamSynchronize(s));
  KC_REQUIRE(hinfo == 0, KC_ENOCONV, "Gram eigen-decomposition did not converge");
  // ascending, column-major (vector j = cm[j*n .. j*n+n)) -> descending, columns of V
  V.assign((size_t)n * n, 0.0);
  w.resize(n);
  for (int c = 0; c < n; ++c) {
    const double* q = &cm[(size_t)(n - 1 - c) * n];
    w[c] = d[n - 1 - c];
    for (int r = 0; r < n; ++r) V[(size_t)r * n + c] = q[r];
  }
}

}  // namespace kc
