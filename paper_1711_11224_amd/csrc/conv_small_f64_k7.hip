// Small-PSF kernel instantiations: double storage, z tap count 7.
#include "conv_small.h"

namespace ndc {
NDC_SMALL_PART(f64_k7, double, 7, 7)
}  // namespace ndc
