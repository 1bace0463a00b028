// Steps (a) and (c) of eq. three-steps for any number of slices N (Section 3.2): the
// diagonalisation C_alpha = V diag(lambda_k) V^{-1}, V = Lambda_alpha^{-1} F_N, turns the
// all-at-once coarse problem into N/2+1 independent spatial problems (the input is real, so
// bins k and N-k are conjugate).  The model problems of Section 5 use N = 24, 25 and 30,
// which are no powers of two; the transforms here are dense sums over the slices with a
// twiddle table (N <= 64, at most 64 x 33 complex products per spatial point), one thread
// per output value so that the loads over the spatial index are coalesced.
#include <cmath>

#include "models.h"
#include "reduce.h"

namespace kc {
namespace {

__global__ __launch_bounds__(256) void slice_dft_kernel(const double* __restrict__ D,
                                                        const int32_t* __restrict__ list, int N, int K,
                                                        int64_t Nx, const double* __restrict__ tw,
                                                        const double* __restrict__ lam, double scale,
                                                        cplx* __restrict__ spec) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  const int64_t li = blockIdx.z;
  if (p >= Nx) return;
  const int64_t m = list ? list[li] : li;
  const double* Dm = D + m * N * Nx + p;
  double re = 0.0, im = 0.0;
  int idx = 0;   // k s mod N
  for (int s = 0; s < N; ++s) {
    const double v = lam[s] * Dm[(int64_t)s * Nx];
    re += tw[2 * idx] * v;        // conj(w^{ks}) = cos - i sin
    im -= tw[2 * idx + 1] * v;
    idx += k;
    if (idx >= N) idx -= N;
  }
  spec[(m * K + k) * Nx + p] = cplx{re * scale, im * scale};
}

// one block row per (sample, slice); maxima by a block reduction and one atomic per block
__global__ __launch_bounds__(256) void slice_idft_kernel(const cplx* __restrict__ spec,
                                                         const int32_t* __restrict__ list, int N, int K,
                                                         int64_t Nx, const double* __restrict__ tw,
                                                         const double* __restrict__ lam, double scale,
                                                         double* __restrict__ U, int accumulate,
                                                         unsigned long long* __restrict__ maxima) {
  __shared__ double red[2 * 4];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  const int64_t li = blockIdx.z;
  const int64_t m = list ? list[li] : li;
  double inc = 0.0, un = 0.0;
  if (p < Nx) {
    const cplx* q = spec + m * K * Nx + p;
    // bins 1 .. ceil(N/2)-1 stand for themselves and their conjugates N-k
    const int kpair = (N - 1) / 2;
    double acc = q[0].re;
    int idx = 0;   // k s mod N
    for (int k = 1; k <= kpair; ++k) {
      idx += s;
      if (idx >= N) idx -= N;
      const cplx v = q[(int64_t)k * Nx];
      acc += 2.0 * (tw[2 * idx] * v.re - tw[2 * idx + 1] * v.im);
    }
    if ((N & 1) == 0) {
      const cplx v = q[(int64_t)(N / 2) * Nx];
      acc += (s & 1) ? -v.re : v.re;
    }
    const double d = acc * scale / lam[s];
    double* u = U + (m * N + s) * Nx + p;
    const double nv = accumulate ? *u + d : d;
    *u = nv;
    inc = fabs(d);
    un = fabs(nv);
  }
  if (maxima) {
    double v[2] = {inc, un};
    const bool mx[2] = {true, true};
    block_reduce<2>(v, mx, red);
    if (threadIdx.x == 0) {
      atomicMax(&maxima[2 * m], (unsigned long long)__double_as_longlong(v[0]));
      atomicMax(&maxima[2 * m + 1], (unsigned long long)__double_as_longlong(v[1]));
    }
  }
}

__global__ __launch_bounds__(256) void slice_error_kernel(const double* __restrict__ U, const double* __restrict__ ref,
                                                          const int32_t* __restrict__ list, int N, int64_t Nx,
                                                          unsigned long long* __restrict__ err) {
  __shared__ double red[4];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  const int64_t li = blockIdx.z;
  const int64_t m = list ? list[li] : li;
  double e = 0.0;
  if (p < Nx) {
    const int64_t o = (m * N + s) * Nx + p;
    e = fabs(U[o] - ref[o]);
  }
  double v[1] = {e};
  const bool mx[1] = {true};
  block_reduce<1>(v, mx, red);
  if (threadIdx.x == 0) atomicMax(&err[m * N + s], (unsigned long long)__double_as_longlong(v[0]));
}

}  // namespace

SliceTables slice_tables(klecgc_ctx* ctx, int N, double alpha, double* d) {
  std::vector<double> h(3 * (size_t)N);
  for (int m = 0; m < N; ++m) {
    const double th = 2.0 * M_PI * (double)m / (double)N;
    h[2 * m] = std::cos(th);
    h[2 * m + 1] = std::sin(th);
    h[2 * (size_t)N + m] = std::pow(alpha, (double)m / (double)N);
  }
  KC_TRY_HIP(hipMemcpyAsync(d, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, ctx->stream));
  KC_TRY_HIP(hipStreamSynchronize(ctx->stream));   // h is released on return
  return SliceTables{d, d + 2 * (size_t)N};
}

void launch_slice_dft(hipStream_t st, const double* D, const int32_t* list, int64_t nlist, int N, int64_t Nx,
                      const SliceTables& tb, cplx* spec) {
  if (nlist <= 0) return;
  const int K = model_bins(N);
  dim3 grid((unsigned)((Nx + 255) / 256), (unsigned)K, (unsigned)nlist);
  slice_dft_kernel<<<grid, 256, 0, st>>>(D, list, N, K, Nx, tb.tw, tb.lam, 1.0 / std::sqrt((double)N), spec);
  KC_LAUNCH_CHECK();
}

void launch_slice_idft(hipStream_t st, const cplx* spec, const int32_t* list, int64_t nlist, int N, int64_t Nx,
                       const SliceTables& tb, double* U, bool accumulate, unsigned long long* maxima) {
  if (nlist <= 0) return;
  const int K = model_bins(N);
  dim3 grid((unsigned)((Nx + 255) / 256), (unsigned)N, (unsigned)nlist);
  slice_idft_kernel<<<grid, 256, 0, st>>>(spec, list, N, K, Nx, tb.tw, tb.lam, 1.0 / std::sqrt((double)N), U,
                                          accumulate ? 1 : 0, maxima);
  KC_LAUNCH_CHECK();
}

void launch_slice_error(hipStream_t st, const double* U, const double* ref, const int32_t* list, int64_t nlist,
                        int N, int64_t Nx, unsigned long long* err) {
  if (nlist <= 0) return;
  dim3 grid((unsigned)((Nx + 255) / 256), (unsigned)N, (unsigned)nlist);
  slice_error_kernel<<<grid, 256, 0, st>>>(U, ref, list, N, Nx, err);
  KC_LAUNCH_CHECK();
}

}  // namespace kc
