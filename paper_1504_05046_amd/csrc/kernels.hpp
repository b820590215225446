// Launch wrappers of the device kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "types.hpp"

namespace bsm {

enum Form : int { FORM_F64 = 0, FORM_F32 = 1, FORM_BF16X3 = 2 };

constexpr int kNoKLimit = 1 << 30;

// Task range of each XCD: tasks begin[x] .. begin[x+1]-1 run on XCD x.
struct XcdMap {
  int32_t begin[kXcds + 1];
};

// Arguments of one tile-kernel launch.
struct TileArgs {
  const Item* items;
  const Triple* tri;
  XcdMap map;
  const ProductArgs* prods;  // per-product operands (batches); NULL = `single` for every task
  ProductArgs single;
  int accumulate;            // C = alpha*AB + C instead of C = alpha*AB (last window only)
  int k_lo, k_hi;            // only triples with k in [k_lo, k_hi) (k-window)
  int win_first, win_last;   // first window starts from 0, later ones from the partial sums
  uint64_t* stamps;          // 2 per task: start/end of the 100 MHz constant clock, or NULL
};

hipError_t launch_tiles_f64(int variant, int64_t grid, const TileArgs& args, hipStream_t stream);
hipError_t launch_tiles_f32(int variant, int64_t grid, const TileArgs& args, hipStream_t stream);

// dst[i] = src[i] rounded to FP32 for i < n.
hipError_t launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t stream);

// Three bf16 slices of every block of one operand (see SplitBlock), planes `plane` elements apart.
hipError_t launch_split_bf16x3(const SplitBlock* blocks, int64_t nblocks, const double* src,
                               uint16_t* dst, int64_t plane, hipStream_t stream);

hipError_t launch_tiles_bf16x3(int variant, int64_t grid, const TileArgs& args, hipStream_t stream);

}  // namespace bsm
