// Launch of the tile kernels: picks the instantiation of a variant and window kind (the
// instantiations live in separate translation units, see kernels_tile.hip and kernels_bf16x3.hip).
#include "kernels.hpp"

namespace bsm {

#define BSM_CASE_F64(ID, TM, TN, KC, NW, OCC)                          \
  case ID:                                                             \
    return args.win_first ? launch_tile_unit_0_##ID##_0(grid, args, stream) \
                          : launch_tile_unit_0_##ID##_1(grid, args, stream);
#define BSM_CASE_F32(ID, TM, TN, KC, NW, OCC)                          \
  case ID:                                                             \
    return args.win_first ? launch_tile_unit_1_##ID##_0(grid, args, stream) \
                          : launch_tile_unit_1_##ID##_1(grid, args, stream);

hipError_t launch_tiles_f64(int variant, int64_t grid, const TileArgs& args, hipStream_t stream) {
  if (grid <= 0) return hipSuccess;
  switch (variant) {
    BSM_TILE_VARIANTS(BSM_CASE_F64)
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_tiles_f32(int variant, int64_t grid, const TileArgs& args, hipStream_t stream) {
  if (grid <= 0) return hipSuccess;
  switch (variant) {
    BSM_TILE_VARIANTS(BSM_CASE_F32)
    default:
      return hipErrorInvalidValue;
  }
}

#define BSM_CASE_B3(ID, TM, TN, KC, NW, OCC)                                         \
  case ID:                                                                         \
    return args.win_first ? launch_b3_unit_##ID##_0(grid, args, stream)            \
                          : launch_b3_unit_##ID##_1(grid, args, stream);

hipError_t launch_tiles_bf16x3(int variant, int64_t grid, const TileArgs& args, hipStream_t stream) {
  if (grid <= 0) return hipSuccess;
  switch (variant) {
    BSM_BF16_VARIANTS(BSM_CASE_B3)
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace bsm
