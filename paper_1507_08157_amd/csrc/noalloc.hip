// Device-resident workspace for the allocation-free operator application
// (tddft_apply_noalloc): a file-scope device array, one copy per GPU, held until the
// process ends.  Its device address is looked up once per device with that device
// current; the array's name in host code is only a host-side stand-in.
#include <mutex>

#include "handle.h"

namespace tddft {

constexpr size_t kScratchBytes = (size_t)256 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

size_t scratch_capacity() { return kScratchBytes; }

// Device address of the current device's copy of the workspace (device must be current).
void *scratch_address(int device) {
  TD_REQUIRE(device >= 0 && device < kMaxDevices, "device index out of range for the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    TD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    TD_REQUIRE(p != nullptr, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

}  // namespace tddft
