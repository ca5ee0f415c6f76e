// qdse_noalloc.hip -- the fixed device workspace of the entry points that
// allocate nothing (qdse_vjp_noalloc): a file-scope device array of
// kScratchDoubles doubles that every GPU the library runs on holds from
// module load until the process ends.
//
// Host code never passes the array's name to a kernel (on the host it is
// only a stand-in for the symbol): the device address is looked up once per
// device with hipGetSymbolAddress, with that device current, and the cached
// pointer is what the kernels receive.
#include "qdse_internal.h"

#include <mutex>

namespace {

constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[qdse::kScratchDoubles];

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

namespace qdse {

hipError_t noalloc_scratch(int device, double** ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace qdse
