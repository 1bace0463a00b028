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

// float64 DPP permutation within each 16-lane row (every lane has a source)
template <int CTRL>
__device__ __forceinline__ double dpp_row_perm(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
// Every lane of a 16-lane row ends with the row's sum (or NaN-keeping maximum): partners by
// quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror, each step combining
// two equal partial results.
__device__ __forceinline__ double row_reduce(double v, bool is_max) {
  double t = dpp_row_perm<0xB1>(v);
  v = is_max ? nanmax(v, t) : v + t;
  t = dpp_row_perm<0x4E>(v);
  v = is_max ? nanmax(v, t) : v + t;
  t = dpp_row_perm<0x141>(v);
  v = is_max ? nanmax(v, t) : v + t;
  t = dpp_row_perm<0x140>(v);
  v = is_max ? nanmax(v, t) : v + t;
  return v;
}
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Reduce K doubles across the work-group: sums for entries with is_max[k] == false,
// maxima otherwise (a NaN anywhere gives NaN).  `slots` is LDS of at least K * (blockDim/64)
// doubles, blockDim <= 1024.  Within each wave by DPP row butterflies, the four row results
// read back as scalars; one slot per wave; after the barrier lanes 0..nw-1 reduce the slots
// the same way.  Every thread returns the same values, held as scalars (fixed order), so
// control decisions taken on them are uniform.  Contains two barriers; `slots` may be reused
// right after return only by the next call (the second barrier protects it).
template <int K>
__device__ __forceinline__ void block_reduce(double (&v)[K], const bool (&is_max)[K],
                                             double* slots) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double x = row_reduce(v[k], is_max[k]);
    const double r0 = readlane_d(x, 0), r1 = readlane_d(x, 16), r2 = readlane_d(x, 32), r3 = readlane_d(x, 48);
    v[k] = is_max[k] ? nanmax(nanmax(r0, r1), nanmax(r2, r3)) : (r0 + r1) + (r2 + r3);
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) slots[k * nw + wave] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double x = lane < nw ? slots[k * nw + lane] : (is_max[k] ? -INFINITY : 0.0);
    v[k] = readlane_d(row_reduce(x, is_max[k]), 0);
  }
  __syncthreads();
}

}  // namespace kc
