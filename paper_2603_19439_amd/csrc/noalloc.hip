// Static device workspace of grest_update_noalloc, the update that allocates nothing.
//
// The buffers an update sizes by its change list -- the copied change arrays, the packed
// (row, column) keys of Delta and their copy grouped by row, the insertion ranks of the
// merge and the two slots of Delta's columns and signs -- are
// allocated by grest_update on demand (they grow with the largest change list seen).  The
// no-allocation variant takes them from one file-scope device array instead, of a fixed
// size that every device the library runs on holds until the process ends.  Every call on
// a device shares that device's array.
#include <mutex>

#include "grest_internal.h"

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// Device address of `scratch` on `device`, looked up once per device with that device
// current (the caller's current device is restored).  The array's name in host code is a
// host-side stand-in, so kernels and copies must use this address.
hipError_t noalloc_scratch(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}
