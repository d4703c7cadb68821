// Fixed device scratch of the allocation-free entry point (noalloc.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace exg {

// bytes of the scratch array each GPU holds (the largest workspace the
// allocation-free entry point accepts)
constexpr size_t kScratchBytes = (size_t)128 << 20;
constexpr int kScratchMaxDevices = 64;

// Device address of the scratch array on `device`, which must be the current
// device; looked up once per device and cached (thread safe).
hipError_t scratch_address(int device, void** out);

}  // namespace exg
