// MFMA correlation kernels (filled in below).
#include "ndc_device.h"
#include "ndc_internal.h"

namespace ndc {

bool mfma_supported(const Geom &, int, int) { return false; }

ConvPlan plan_conv_mfma(const Geom &, int, int) {
  ConvPlan pl{};
  return pl;
}

hipError_t launch_conv_mfma(const ConvPlan &, const Geom &, int, int, const void *, const void *, void *,
                            const Epi &, hipStream_t) {
  return hipErrorInvalidValue;
}

}  // namespace ndc
