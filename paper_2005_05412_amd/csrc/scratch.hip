// Library-held device memory for runs that must not allocate: one static
// array per GPU, addressed through hipGetSymbolAddress (the array's name in
// host code is a host-side stand-in, not a device address).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "scratch.hpp"

namespace mb {
namespace {

// group tables of one run: simulation descriptors, tile table and neighbour
// flags; each GPU the library runs on holds its own copy until the process ends
constexpr size_t kScratchBytes = size_t(1) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};

__global__ void k_fill_u32(uint32_t *p, size_t n, uint32_t v) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

size_t scratch_capacity() { return kScratchBytes; }

void *scratch_address(int device, std::string &err) {
  if (device < 0 || device >= kMaxDevices) {
    err = "device index out of range for the static scratch";
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_addr[device]) {
    // the device is current (the caller set it); its copy of the array
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return nullptr;
    }
    g_addr[device] = p;
  }
  return g_addr[device];
}

hipError_t fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const unsigned threads = 256;
  const unsigned blocks = unsigned((n + threads - 1) / threads);
  k_fill_u32<<<blocks, threads, 0, st>>>(p, n, v);
  return hipGetLastError();
}

}  // namespace mb
