// Operand conversion for the reduced-precision forms (HBM-bound elementwise pass over the packed
// tiles; the packed layout is kept, only the element type changes).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace bsm {

// dst[i] = src[i] rounded to FP32 (round to nearest even).
__global__ __launch_bounds__(256) void to_f32(const double* __restrict__ src,
                                              float* __restrict__ dst, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = float(src[i]);
}

hipError_t launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 256 * 16) blocks = 256 * 16;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(to_f32, dim3(uint32_t(blocks)), dim3(256), 0, stream, src, dst, n);
  return hipGetLastError();
}

}  // namespace bsm
