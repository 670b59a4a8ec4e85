// The batch table of pic_step_batch_noalloc: a file-scope device array, one
// per GPU the library runs on (held until the process ends), so a caller
// that cannot allocate memory can still advance a batch of runs.  Host code
// reaches it only through the address hipGetSymbolAddress returns on each
// device (the array's name is a host-side stand-in, not a device address).
#include <hip/hip_runtime.h>

#include <mutex>

#include "launch.hpp"
#include "pic_dev.hpp"

namespace pic {

static __device__ __align__(256) BatchTable scratch;

namespace {
constexpr int MAX_DEVICES = 16;
BatchTable* g_scratch_ptr[MAX_DEVICES];
std::mutex g_scratch_mutex;
}  // namespace

hipError_t batch_scratch(BatchTable** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {  // once per device, with that device current
    BatchTable* ptr = nullptr;
    e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace pic
