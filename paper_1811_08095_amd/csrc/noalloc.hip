// Scratch memory of the allocation-free operator application.
//
// odwf_apply_noalloc runs the kernels of odwf_apply with its packed half
// fields carved from one file-scope device array instead of the solver's
// workspace, so that the call itself allocates no device memory (for callers
// under HIP graph capture, in tight serving loops, or in harnesses that forbid
// hipMalloc).  The array is a per-device symbol: every GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// never uses the array's name as a device address; its address on a device is
// resolved once, with that device current, when the first lattice is created
// on it, and kept here.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/odwf.h"
#include "runtime.h"

namespace odwf {

static __device__ __align__(256) unsigned char scratch[ODWF_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_noalloc_mtx;
static void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// Resolve the scratch array's address on `device` (which must be current).
hipError_t noalloc_init(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_noalloc_mtx);
  if (g_noalloc_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_noalloc_ptr[device] = p;
  return hipSuccess;
}

// The device address of the scratch array on `device`, or null before
// noalloc_init ran there.
void* noalloc_scratch(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_noalloc_mtx);
  return g_noalloc_ptr[device];
}

}  // namespace odwf
