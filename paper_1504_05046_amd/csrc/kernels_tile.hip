// One instantiation of the FP64/FP32 tile kernel per translation unit, so that the build compiles
// them in parallel: BSM_UNIT_FORM (0 = FP64, 1 = FP32), BSM_UNIT_ID (variant row) and
// BSM_UNIT_RESUME (0 = first k-window, 1 = a later one) are set on the compiler's command line.
// Without them this unit is empty.
#include "tile_impl.hpp"

#if defined(BSM_UNIT_FORM) && defined(BSM_UNIT_ID) && defined(BSM_UNIT_RESUME)
#define BSM_UNIT_NAME3(F, I, R) launch_tile_unit_##F##_##I##_##R
#define BSM_UNIT_NAME(F, I, R) BSM_UNIT_NAME3(F, I, R)

namespace bsm {
hipError_t BSM_UNIT_NAME(BSM_UNIT_FORM, BSM_UNIT_ID, BSM_UNIT_RESUME)(int64_t grid,
                                                                     const TileArgs& args,
                                                                     hipStream_t stream) {
  return launch_tile_instance<BSM_UNIT_ID, BSM_UNIT_FORM, BSM_UNIT_RESUME != 0>(grid, args, stream);
}
}  // namespace bsm
#endif
