// Small-PSF kernel instantiations: float storage, z tap counts 1 and 3.
#include "conv_small.h"

namespace ndc {
NDC_SMALL_PART(f32_k13, float, 1, 3)
}  // namespace ndc
