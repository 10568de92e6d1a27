// wave_scratch.cpp -- the static device workspace of wave_forward_noalloc.
//
// A file-scope device array, one copy per device that loads the library (held until
// the process ends), shared by every wave_forward_noalloc call on that device. In
// host code `scratch` only names the symbol; its address on a device comes from
// hipGetSymbolAddress, taken once per device with that device current, and that
// address is what the kernels receive as their workspace.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/wave.h"
#include "wave_host.h"

namespace wave {

constexpr int kMaxScratchDevices = 64;
__device__ __align__(256) char scratch[kScratchBytes];

int scratch_address(void** out) {
  static std::mutex mu;
  static void* addr[kMaxScratchDevices] = {};
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices) return WAVE_EDEVICE;
  std::lock_guard<std::mutex> lk(mu);
  if (addr[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
      return WAVE_EDEVICE;
    addr[dev] = p;
  }
  *out = addr[dev];
  return WAVE_OK;
}

}  // namespace wave
