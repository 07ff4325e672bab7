// conv_dH_nd_noalloc: the PSF gradient with its split-K partials in a
// file-scope device array instead of a caller workspace, for callers that
// cannot allocate device memory.
//
// `scratch` below is a device symbol.  In host code its name is only a
// host-side stand-in: its device address is looked up once per device with
// hipGetSymbolAddress (each GPU holds its own copy of the array) and only
// that address is ever handed to kernels.
#include <mutex>

#include "ndc_internal.h"

namespace {

constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[NDC_DH_SCRATCH_BYTES];

std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices];  // device address of `scratch` per device (null: not looked up yet)

// Device address of the current device's scratch array (null on failure).
void *current_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    scratch_ptr[dev] = ptr;
  }
  return scratch_ptr[dev];
}

}  // namespace

extern "C" int conv_dH_nd_noalloc(int n, const int64_t *m, const int64_t *p, const void *X, const void *G, void *dH,
                                  int dtype, void *stream) {
  return ndc::dH_checked(n, m, p, X, G, dH, dtype, nullptr, 0, NDC_DH_SCRATCH_BYTES, current_scratch, stream);
}
