// Launch wrappers of the device kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "types.hpp"

namespace bsm {

// Task range of each XCD: tasks begin[x] .. begin[x+1]-1 run on XCD x.
struct XcdMap {
  int32_t begin[kXcds + 1];
};

hipError_t launch_f64(int variant, int64_t grid, const Item* items, const Triple* tri,
                      const XcdMap& map, const ProductArgs* prods, const ProductArgs& single,
                      int accumulate, hipStream_t stream);

}  // namespace bsm
