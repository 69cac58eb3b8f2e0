// Host-side helpers shared by the C-ABI entry points: error state, problem
// validation, creation of one job's device state, and the combination of
// iterations into one estimate.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "mcv.h"
#include "mcv_internal.h"

namespace mcv {

// Records msg as the calling thread's last error and returns st.
mcv_status fail(mcv_status st, const std::string& msg);
const char* last_error();

#define MCV_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ::mcv::fail(MCV_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

mcv_status validate_problem(const mcv_problem* p);

// Device memory of the library: from the allocator installed with
// mcv_set_allocator, else hipMalloc.  Each block goes back to the allocator
// that made it.  dev_free waits for the device first (as hipFree does), so a
// caching allocator never hands out memory that queued work still reads.
hipError_t dev_alloc(void** p, size_t bytes);
void dev_free(void* p);
mcv_status set_allocator(mcv_alloc_fn alloc, mcv_free_fn release, void* ctx);

// The static work area of mcv_unweight_noalloc on `device` (noalloc.hip):
// its device address, looked up once per device with that device current,
// and its size.
mcv_status static_work_area(int device, char** out);
size_t static_work_bytes();

// Compute units of the current device.
mcv_status device_cus(int* device, int* n_cu);

// Creates one job's device state in a single device block (*block, freed with
// hipFree): problem arrays, derived constants, equidistant grids, tables,
// allocation and pass buffers, history, and the job's device record
// (j->self).  Per-unit partial buffers are carved for gmax work units when
// gmax > 0 and left null otherwise.  Synchronises `s` before returning.
mcv_status job_create(const mcv_problem* p, int gmax, int64_t n_points, int n_cu, hipStream_t s,
                      JobDev* j, void** block);

// Device bytes job_create would allocate for this problem (a valid one).
size_t job_block_bytes(const mcv_problem* p, int gmax);

// Bytes of the per-unit partial buffers of a job for G work units.
size_t partial_bytes(const JobDev& j, int G);
// Points the job's partial buffers into `base` (partial_bytes(j, G) bytes).
void carve_partials(JobDev& j, int G, char* base);

// Inverse-variance weighted mean of history rows [first, n) (kHistStride
// doubles each), its error and chi^2/ndf; iterations with zero error are
// exact and are averaged alone.
void combine_history(const double* hist, int n, int first, mcv_summary* out);

}  // namespace mcv
