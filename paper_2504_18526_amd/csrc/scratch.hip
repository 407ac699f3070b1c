// Fixed device scratch of the library: one statically sized array per GPU,
// for the entry point that allocates nothing (helmholtz_solve_noalloc).
//
// The array is a device symbol: its host-side name is not a device address.
// Its address on a device is taken once per device, with that device current,
// by hipGetSymbolAddress, and every later use (kernel arguments, clears)
// goes through that address.  Each GPU holds its own copy until the process
// ends.  Calls that use it on one GPU share it, so calls that overlap on one
// GPU race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "scratch.hpp"

namespace sisdc {

namespace {

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kScratchDevices] = {};

__global__ void k_zero_words(double* __restrict__ p, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = 0.0;
}

}  // namespace

hipError_t scratch_region(int dev, void** ptr) {
  if (!ptr || dev < 0 || dev >= kScratchDevices) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev) return hipErrorInvalidDevice;  // the address is taken with that device current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_zero_scratch(void* p, size_t bytes, hipStream_t s) {
  const long n = (long)(bytes / sizeof(double));
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<long>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_zero_words, dim3(blocks), dim3(256), 0, s, (double*)p, n);
  return hipGetLastError();
}

}  // namespace sisdc
