// Small-PSF kernel instantiations: double storage, z tap count 5.
#include "conv_small.h"

namespace ndc {
NDC_SMALL_PART(f64_k5, double, 5, 5)
}  // namespace ndc
