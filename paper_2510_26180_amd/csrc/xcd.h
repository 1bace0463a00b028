// Work-group placement on the MI355X's 8 XCDs.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace kc {

constexpr int kXcds = 8;

// The dispatcher deals the work-groups of a launch to the XCDs in turn (work-group b runs
// on XCD b % 8), and each XCD has its own L2.  xcd_major maps work-group b of G to an item
// index such that XCD x takes a contiguous range of items (the first G % 8 XCDs one item
// more than the rest), so consecutive items, e.g. systems that share a coefficient field,
// run under one L2.  A bijection of [0, G).
__device__ __forceinline__ int64_t xcd_major(int64_t b, int64_t G) {
  const int64_t base = G / kXcds, extra = G % kXcds;
  const int64_t x = b % kXcds, k = b / kXcds;
  return (x < extra ? x * (base + 1) : extra * (base + 1) + (x - extra) * base) + k;
}

}  // namespace kc
