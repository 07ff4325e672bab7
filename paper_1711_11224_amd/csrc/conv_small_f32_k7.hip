// Small-PSF kernel instantiations: float storage, z tap count 7.
#include "conv_small.h"

namespace ndc {
NDC_SMALL_PART(f32_k7, float, 7, 7)
}  // namespace ndc
