// Work-group reductions for 64-wide wavefronts (gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace kc {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// max that keeps NaN (fmax would drop it): once NaN, always NaN
__device__ __forceinline__ double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }
__device__ __forceinline__ double wave_nanmax(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = nanmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Reduce K doubles across the work-group: sums for entries with is_max[k] == false,
// maxima otherwise.  `slots` is LDS of at least K * (blockDim/64) doubles.  Every
// thread returns the same values (fixed summation order), so control decisions
// taken on them are uniform.  Contains two barriers; `slots` may be reused right
// after return only by the next call (the second barrier protects it).
template <int K>
__device__ __forceinline__ void block_reduce(double (&v)[K], const bool (&is_max)[K],
                                             double* slots) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = is_max[k] ? wave_nanmax(v[k]) : wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) slots[k * nw + wave] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double acc = slots[k * nw];
    for (int w = 1; w < nw; ++w) acc = is_max[k] ? nanmax(acc, slots[k * nw + w]) : acc + slots[k * nw + w];
    v[k] = acc;
  }
  __syncthreads();
}

}  // namespace kc
