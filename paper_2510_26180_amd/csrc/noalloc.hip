// The device scratch array behind the allocation-free entry point fine_propagate_noalloc,
// for callers that cannot allocate device memory (code under graph capture, serving loops,
// harnesses that forbid hipMalloc).
//
// `scratch` is a file-scope device array of kScratchBytes; every GPU the library runs on
// holds its own copy until the process ends.  In host code its name is only a stand-in:
// its device address is resolved once per device with hipGetSymbolAddress (at context
// creation, with that device current) and only that address is ever handed to kernels or
// runtime calls.  All calls on one GPU share the array and it keeps the last call's
// contents: what must start at zero is cleared by the call that uses it, and calls that
// overlap on one GPU race.
#include <algorithm>
#include <map>
#include <mutex>

#include "common.h"

namespace kc {

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per GPU

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;   // device -> address of its copy of `scratch`

__global__ void zero_words_kernel(unsigned int* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

}  // namespace

hipError_t scratch_resolve(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) {
    *out = nullptr;
    return e != hipSuccess ? e : hipErrorInvalidSymbol;
  }
  g_scratch_addr[device] = ptr;
  *out = ptr;
  return hipSuccess;
}

size_t scratch_bytes() { return kScratchBytes; }

// Clears `bytes` (a multiple of 4) at p with a kernel rather than a memset node, so the
// clear may sit inside a caller's graph capture.
void launch_zero_bytes(hipStream_t s, void* p, size_t bytes) {
  const int64_t n = (int64_t)(bytes / 4);
  const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024));
  zero_words_kernel<<<blocks, 256, 0, s>>>((unsigned int*)p, n);
  KC_LAUNCH_CHECK();
}

}  // namespace kc
