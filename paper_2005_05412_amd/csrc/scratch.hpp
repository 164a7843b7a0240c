// The library's static device scratch (scratch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace mb {

// The static device scratch of this GPU (the device must be current): its
// address (looked up once per device with hipGetSymbolAddress), or null with a
// message; its size in bytes.  Shared by every call on that GPU.
void *scratch_address(int device, std::string &err);
size_t scratch_capacity();
// p[0..n) = v on st (a small kernel, not a memset)
hipError_t fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t st);

}  // namespace mb
