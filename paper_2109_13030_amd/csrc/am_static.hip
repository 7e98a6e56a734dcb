// am_static.hip -- the library's static device table for the multi-problem
// launch that allocates nothing (am_solve_multi_static).
//
// `scratch` holds the problem table of one such launch: up to
// AM_STATIC_MAX_PROBLEMS descriptors.  Every GPU the library runs on holds
// its own copy of the array until the process ends.  Host code never passes
// the array's name to a kernel or a copy (on the host it is a stand-in, not
// a device address): the device address of each GPU's copy is looked up
// once, with that GPU current, and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "am_internal.h"

namespace amk {
namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[AM_STATIC_MAX_PROBLEMS * sizeof(Desc)];

std::mutex g_mu;
Desc *g_table[kMaxDevices] = {};

}  // namespace

hipError_t static_table(int device, Desc **out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_table[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // looked up with that device current only
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_table[device] = static_cast<Desc *>(p);
  }
  *out = g_table[device];
  return hipSuccess;
}

}  // namespace amk
