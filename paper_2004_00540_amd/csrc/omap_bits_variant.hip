// One bit-sliced variant: k_bits instantiated for OMAP_BITS_T layers per
// visit, and its launch functions (the build compiles this file once per
// variant).
#include "omap_bits.h"

#if !defined(OMAP_BITS_T)
#error "define OMAP_BITS_T"
#endif

namespace omap {

OMAP_DEFINE_BITS_VARIANT(OMAP_BITS_T)

}  // namespace omap
