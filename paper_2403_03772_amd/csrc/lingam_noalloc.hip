// Scratch memory of lingam_causal_order_noalloc: the workspace of an ordering
// held in one file-scope device array, so that the call allocates nothing.
//
// Each GPU the library runs on holds its own copy of `scratch` (its module's
// global memory) until the process ends.  Host code never passes the array's
// name to a kernel or a copy (on the host that name is only a stand-in): the
// device address is looked up once per device with hipGetSymbolAddress, with
// that device current, and cached.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "../../include/lingam.h"
#include "lingam_internal.h"

namespace {

static __device__ __align__(256) char scratch[LINGAM_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device; nullptr until looked up

}  // namespace

namespace lg {

hipError_t noalloc_scratch(int dev, void** ptr) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_ptr[(size_t)dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[(size_t)dev] = p;
  }
  *ptr = g_scratch_ptr[(size_t)dev];
  return hipSuccess;
}

}  // namespace lg
