// Static work area of mcv_unweight_noalloc: a file-scope device array, so
// that entry point needs no device allocation.  Every GPU the library runs
// on holds its own copy until the process ends.  In host code the array's
// name only stands for the symbol; its device address is looked up once per
// device (hipGetSymbolAddress, with that device current) and only that
// address is ever passed to kernels or copies.  Calls that overlap on one
// device share the array and race.  Nothing in it needs clearing: each
// unweighting batch writes its accept flags, weights, points and compaction
// records before reading them.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "mcv_host.h"

namespace {
constexpr size_t kScratchBytes = (size_t)8 << 20;  // 8 MiB per device
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace mcv {

namespace {
std::mutex g_mu;
std::map<int, char*> g_addr;  // device ordinal -> device address of `scratch`
}  // namespace

size_t static_work_bytes() { return kScratchBytes; }

mcv_status static_work_area(int device, char** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_addr.find(device);
  if (it != g_addr.end()) {
    *out = it->second;
    return MCV_OK;
  }
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess || cur != device)
    return fail(MCV_E_INVALID, "the static work area is looked up on the current device");
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(MCV_E_DEVICE,
                std::string("address of the static work area: ") + hipGetErrorString(e));
  g_addr[device] = static_cast<char*>(ptr);
  *out = static_cast<char*>(ptr);
  return MCV_OK;
}

}  // namespace mcv
