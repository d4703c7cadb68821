// Fixed device scratch of the allocation-free entry point
// (exageo_loglik_grad_noalloc): a file-scope device array that the code
// object reserves on every GPU the library runs on, for the life of the
// process.  Its device address is looked up once per device, with that device
// current, by the context's creation (exageo_create); host code then uses
// only that address (kernel arguments, copies), never the array's name, which
// on the host is a stand-in and not a device address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "noalloc.h"

namespace {

static __device__ __align__(256) unsigned char scratch[exg::kScratchBytes];

std::mutex g_mu;
void* g_addr[exg::kScratchMaxDevices] = {};

}  // namespace

namespace exg {

hipError_t scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kScratchMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_addr[device] = p;
  }
  *out = g_addr[device];
  return hipSuccess;
}

}  // namespace exg
