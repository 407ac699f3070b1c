// Fixed per-GPU device scratch (scratch.hip) of the entry point that
// allocates nothing.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>

namespace sisdc {

// Size of the static scratch array on every GPU the library runs on.
constexpr size_t kScratchBytes = size_t(32) << 20;

// Device address of the scratch array on device `dev`, which must be the
// current device on the first call for that device (the address is looked up
// then, once, and kept).  hipErrorInvalidDevice if another device is current
// at that first call.
hipError_t scratch_region(int dev, void** ptr);

// Zero `bytes` (a multiple of 8) at device address p with a fill kernel on s.
hipError_t launch_zero_scratch(void* p, size_t bytes, hipStream_t s);

}  // namespace sisdc
