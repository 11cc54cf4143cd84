// One tile-sweep variant: the kernels of omap_sweep.h instantiated for
// OMAP_T layers per visit and OMAP_C columns per lane, and their launch
// functions (the build compiles this file once per variant, in parallel).
#include "omap_sweep.h"
#include "omap_sweep_split.h"

#if !defined(OMAP_T) || !defined(OMAP_C)
#error "define OMAP_T and OMAP_C"
#endif

namespace omap {

OMAP_DEFINE_SWEEP_VARIANT(OMAP_T, OMAP_C)
#if OMAP_C == 1 && OMAP_T == 16
OMAP_DEFINE_SWEEP_SPLIT(OMAP_T)
#endif

}  // namespace omap
