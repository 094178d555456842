// helm_apply_static: helm_apply without any allocation, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).  Every buffer the sweep
// needs beyond its input and output (slab iterates, received layers, exchange words) lives in
// a file-scope device array of kStaticScratchBytes, which each GPU the library runs on holds
// until the process ends.  The sweep processes the right-hand sides in chunks that fit in it.
#include <map>
#include <mutex>

#include "common.h"

namespace {

constexpr size_t kStaticScratchBytes = 128u << 20;

// The array's name is a host-side stand-in, not a device address: host code uses the address
// hipGetSymbolAddress gives for the current device (one copy per GPU), never the name.
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

struct DeviceScratch {
  void* ptr = nullptr;
  unsigned long long seq = 0;   // exchange tags of every call on this GPU (monotonic)
};
std::mutex g_mu;
std::map<int, DeviceScratch> g_dev;

}  // namespace

extern "C" int helm_apply_static(helm_handle* h, const void* r_dev, void* z_dev, int R, int adjoint,
                                 void* stream) {
  if (!h) {
    set_error("handle is NULL");
    return HELM_EINVAL;
  }
  if (!r_dev || !z_dev || r_dev == z_dev || R < 1) {
    set_error("need non-NULL, non-aliasing vectors and R >= 1");
    return HELM_EINVAL;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    set_error("hipGetDevice failed");
    return HELM_EHIP;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceScratch& d = g_dev[dev];
  if (!d.ptr) {
    // once per device, with that device current
    const hipError_t e = hipGetSymbolAddress(&d.ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !d.ptr) {
      d.ptr = nullptr;
      set_error(std::string("hipGetSymbolAddress of the static scratch: ") + hipGetErrorString(e));
      return HELM_EHIP;
    }
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  FixedScratch fx{static_cast<char*>(d.ptr), kStaticScratchBytes, &d.seq};
  const hipError_t e = launch_apply_fixed(h, r_dev, z_dev, R, adjoint != 0, fx, s);
  if (e == hipErrorOutOfMemory) {
    set_error("one right-hand side's sweep scratch exceeds the static scratch of " +
              std::to_string(kStaticScratchBytes) + " bytes");
    return HELM_EINVAL;
  }
  if (e != hipSuccess) {
    set_error(std::string("static sweep launch: ") + hipGetErrorString(e));
    return HELM_EHIP;
  }
  return HELM_OK;
}
