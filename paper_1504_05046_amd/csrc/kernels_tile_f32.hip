// FP32 instantiation of the tile kernels.
#include "tile_impl.hpp"

namespace bsm {
hipError_t launch_tiles_f32(int variant, int64_t grid, const TileArgs& args, hipStream_t stream) {
  if (grid <= 0) return hipSuccess;
  return launch_tiles_form<FORM_F32>(variant, grid, args, stream);
}
}  // namespace bsm
