// Device scratch of the entry point that allocates nothing (cbc_apply_noalloc).
//
// The array below is the workspace of cbc_apply_noalloc: the offset tables of the call's plan and
// the environments and per-step scratch that cbc_apply keeps in the caller's workspace. Every GPU
// the library runs on holds one copy for the life of the process. Host code never passes the
// array's name to a kernel or a copy (on the host it is only a stand-in for the symbol); it asks
// the runtime for the array's address on each device once, with that device current, and uses
// that address.
#include <mutex>

#include "cbc_internal.h"

namespace cbc {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEV = 64;
std::mutex g_mu;
void* g_addr[NOALLOC_MAX_DEV] = {};
}  // namespace

hipError_t noalloc_scratch(void** ptr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= NOALLOC_MAX_DEV) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_addr[dev] = p;
  }
  *ptr = g_addr[dev];
  return hipSuccess;
}

}  // namespace cbc
