// Library-owned device scratch for the entry point that allocates nothing
// (mppi_step_noalloc): one solve's device block (descriptor, request data,
// folded latents, tile partials, costs, weights, result) and, on the fused
// path, its launch block (descriptor, tile list, work counter) are placed in
// this file-scope array instead of the engine's pool.
//
// Each device the library runs on holds its own copy of the array for the
// life of the process.  Host code never uses the array's name as a device
// address: scratch_device_address() looks the address up once per device,
// with that device current, and every later use goes through that pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"

namespace mppi {

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_lookup_mu;
void* g_addr[kMaxDevices] = {};
std::mutex g_use_mu[kMaxDevices];
}  // namespace

hipError_t scratch_device_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_lookup_mu);
  if (!g_addr[device]) {
    // the caller has made `device` current
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_addr[device] = p;
  }
  *out = g_addr[device];
  return hipSuccess;
}

std::mutex& scratch_use_mutex(int device) { return g_use_mu[device < 0 || device >= kMaxDevices ? 0 : device]; }

}  // namespace mppi
