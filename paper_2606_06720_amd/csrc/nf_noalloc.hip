// Fixed device workspace of the allocation-free pressure solve
// (nf_pressure_solve_noalloc in include/nf.h).
//
// The workspace is one file-scope device array of NOALLOC_SCRATCH_BYTES; every
// GPU the library runs on holds its own copy until the process ends.  Host
// code never uses the array's name as an address: the device address of each
// GPU's copy is looked up once, with that GPU current, and kept per device.
// Calls on one GPU share its copy, so calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "nf_internal.h"

namespace nf {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex scratch_mu;
void* scratch_dev[NOALLOC_MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch(void** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    scratch_dev[dev] = ptr;
  }
  *out = scratch_dev[dev];
  return hipSuccess;
}

}  // namespace nf
