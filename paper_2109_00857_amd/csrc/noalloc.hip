// Scratch of the allocation-free value iteration (mdp_value_iterate_noalloc):
// a static device array of MDP_NOALLOC_SCRATCH_BYTES, one copy per GPU, held
// from the library's load until the process ends. Host code never passes the
// array's name to a kernel or a copy (on the host it is only a stand-in
// symbol): the context's set-up asks the runtime once per device for that
// device's copy's address and every later use goes through that pointer.
#include <mutex>

#include "mdp_internal.h"

static __device__ __align__(256) unsigned char scratch[MDP_NOALLOC_SCRATCH_BYTES];

namespace mdpk {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(int device, void **out)
{
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_addr[device] = p;
  }
  *out = g_addr[device];
  return hipSuccess;
}

}  // namespace mdpk
