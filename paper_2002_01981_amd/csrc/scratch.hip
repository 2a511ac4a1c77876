// scratch.hip -- the device memory of ifcm_solve_noalloc, the entry point
// that allocates nothing.
//
// Callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc) get a solve whose whole
// workspace -- g_inv, the second membership buffer of the Jacobi iteration,
// the tile sums, the solve state, the launch tables, the objective history
// and the check flags -- lives in one file-scope device array.  Every GPU the
// library runs on holds its own copy of the array (kScratchBytes) until the
// process ends.
//
// On the host, `scratch` names a host-side stand-in, not device memory: its
// device address is taken once per device with hipGetSymbolAddress, with
// that device current, and only that address is ever handed to kernels or
// copies.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pifcm_kernels.h"

namespace pifcm {

namespace {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_addr_mu;
void* g_addr[kMaxDevices] = {};
std::mutex g_call_mu[kMaxDevices];

}  // namespace

hipError_t scratch_region(int device, void** ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_addr_mu);
  if (!g_addr[device]) {
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return e;
    if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return e;
    g_addr[device] = p;
  }
  *ptr = g_addr[device];
  return hipSuccess;
}

std::mutex* scratch_call_lock(int device) {
  return device >= 0 && device < kMaxDevices ? &g_call_mu[device] : nullptr;
}

}  // namespace pifcm
