// Small-PSF kernel instantiations: float storage, z tap count 5.
#include "conv_small.h"

namespace ndc {
NDC_SMALL_PART(f32_k5, float, 5, 5)
}  // namespace ndc
