// Library-owned device scratch for callers that cannot allocate (aux_solve_batched_noalloc).
//
// `scratch` is a file-scope device array: every GPU the library runs on holds its own copy, at
// its own address, from the moment the code object is loaded until the process ends.  In host
// code the array's name is only a host-side stand-in, so its device address is looked up once
// per device with hipGetSymbolAddress (with that device current) and kept; every kernel
// argument and every copy uses that address.  All calls on one device share the array: calls
// that overlap on one device race.
#include <mutex>

#include "common.h"

namespace dpm {

namespace {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

dpm_status static_scratch(void** out) {
  int dev = 0;
  DPM_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d beyond the %d devices the static scratch tracks", dev, kMaxDevices);
    return DPM_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
      return DPM_EHIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DPM_OK;
}

}  // namespace dpm
