// Small-PSF kernel instantiations: double storage, z tap counts 1 and 3.
#include "conv_small.h"

namespace ndc {
NDC_SMALL_PART(f64_k13, double, 1, 3)
}  // namespace ndc
