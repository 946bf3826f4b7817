// Device scratch array of the allocation-free V-cycle (dgmg_scratch.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace dgmg {

// Size of the per-device scratch array: the largest set of coarse-level
// vectors dgmg_vcycle_noalloc accepts.
constexpr size_t kScratchBytes = size_t(64) << 20;

// Device address of the scratch array on the current device (looked up with
// hipGetSymbolAddress on the first call per device, then cached).
hipError_t scratch_address(void** ptr);

}  // namespace dgmg
