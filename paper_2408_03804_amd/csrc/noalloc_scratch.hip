// Scratch of the allocation-free projection (fft_homog_project_noalloc): the twiddle tables and
// the half spectrum.  A file-scope device array: every device the library runs on holds its own
// copy from module load until the process ends.  Host code never uses the array's name as an
// address (on the host it is only a stand-in); it uses the per-device address that
// hipGetSymbolAddress returns, looked up on the first call with that device current.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.h"

namespace fh {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices];  // address of `scratch` on each device, once looked up
}  // namespace

hipError_t noalloc_scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace fh
