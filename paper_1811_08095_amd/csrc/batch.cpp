// Batch engine (continuous batching at CG-iteration granularity).
#include "runtime.h"

using namespace odwf;

extern "C" odwf_status odwf_batch_create(odwf_solver, int, odwf_prec, odwf_batch*) {
  set_error("odwf_batch_create: not available");
  return ODWF_EINVAL;
}
extern "C" odwf_status odwf_batch_admit(odwf_batch, const void*, double, double, int, int*, void*) { return ODWF_EINVAL; }
extern "C" odwf_status odwf_batch_step(odwf_batch, int, void*) { return ODWF_EINVAL; }
extern "C" odwf_status odwf_batch_poll(odwf_batch, int, int*, odwf_stats*, void*) { return ODWF_EINVAL; }
extern "C" odwf_status odwf_batch_retire(odwf_batch, int, void*, odwf_stats*, void*) { return ODWF_EINVAL; }
extern "C" odwf_status odwf_batch_free_slots(odwf_batch, int*) { return ODWF_EINVAL; }
extern "C" void odwf_batch_destroy(odwf_batch) {}
