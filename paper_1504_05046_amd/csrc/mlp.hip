// Task cost model: a 5 -> 32 -> 32 -> 1 ReLU network (FP32) that predicts a task's log run time
// from its features, trained with Adam on timings the multiply itself records.
//
// Parameter layout (shared with the host side): W1 (32 x 5, row-major), b1 (32), W2 (32 x 32,
// row-major), b2 (32), w3 (32), b3 (1).
//
// Training reductions are deterministic: every workgroup reduces its chunk of samples in a fixed
// order into its own row of partial sums, and a second kernel adds the rows in workgroup order.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace bsm {

namespace {

constexpr int F = kMlpIn, H = kMlpHidden;
constexpr int OW1 = 0, OB1 = OW1 + H * F, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H,
              OB3 = OW3 + H;
static_assert(OB3 + 1 == kMlpParams, "parameter layout");
constexpr int CHUNK = 256;  // samples per workgroup in the training kernels

// forward of one sample; fills the pre-activations z1, z2 and returns y
__device__ inline float forward1(const float* __restrict__ p, const float* x, float* z1, float* z2) {
  float h1[H];
#pragma unroll
  for (int u = 0; u < H; ++u) {
    float s = p[OB1 + u];
#pragma unroll
    for (int f = 0; f < F; ++f) s += p[OW1 + u * F + f] * x[f];
    z1[u] = s;
    h1[u] = s > 0.f ? s : 0.f;
  }
  float y = p[OB3];
#pragma unroll 4
  for (int u = 0; u < H; ++u) {
    float s = p[OB2 + u];
#pragma unroll
    for (int q = 0; q < H; ++q) s += p[OW2 + u * H + q] * h1[q];
    z2[u] = s;
    y += p[OW3 + u] * (s > 0.f ? s : 0.f);
  }
  return y;
}

__global__ __launch_bounds__(256) void mlp_forward(const float* __restrict__ params,
                                                   const float* __restrict__ X, int64_t n,
                                                   float* __restrict__ Y, MlpNorm norm) {
  __shared__ float p[kMlpParams];
  for (int q = threadIdx.x; q < kMlpParams; q += blockDim.x) p[q] = params[q];
  __syncthreads();
  for (int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; b < n;
       b += int64_t(gridDim.x) * blockDim.x) {
    float x[F], z1[H], z2[H];
#pragma unroll
    for (int f = 0; f < F; ++f) x[f] = (X[b * F + f] - norm.fmean[f]) / norm.fstd[f];
    Y[b] = forward1(p, x, z1, z2) * norm.tstd + norm.tmean;
  }
}

__global__ __launch_bounds__(256) void mlp_normalize(float* __restrict__ X, float* __restrict__ T,
                                                     int64_t n, MlpNorm norm) {
  for (int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; b < n;
       b += int64_t(gridDim.x) * blockDim.x) {
#pragma unroll
    for (int f = 0; f < F; ++f) X[b * F + f] = (X[b * F + f] - norm.fmean[f]) / norm.fstd[f];
    T[b] = (T[b] - norm.tmean) / norm.tstd;
  }
}

// One workgroup per chunk of CHUNK samples: per-sample forward and backward into LDS, then the
// chunk's gradient and loss partial sums (samples added in index order).
__global__ __launch_bounds__(CHUNK) void mlp_grad_partial(const float* __restrict__ params,
                                                          const float* __restrict__ X,
                                                          const float* __restrict__ T, int64_t n,
                                                          float inv_n, float* __restrict__ part,
                                                          float* __restrict__ part_loss) {
  __shared__ float p[kMlpParams];
  __shared__ float sx[CHUNK][F];
  __shared__ float sh1[CHUNK][H + 1];
  __shared__ float sd1[CHUNK][H + 1];
  __shared__ float sd2[CHUNK][H + 1];
  __shared__ float sh2[CHUNK][H + 1];
  __shared__ float sdy[CHUNK];
  __shared__ float sl[CHUNK];
  for (int q = threadIdx.x; q < kMlpParams; q += blockDim.x) p[q] = params[q];
  __syncthreads();
  const int64_t b0 = int64_t(blockIdx.x) * CHUNK;
  const int tl = threadIdx.x;
  const int64_t b = b0 + tl;
  const int cnt = int(min(int64_t(CHUNK), n - b0));
  if (tl < cnt) {
    float x[F], z1[H], z2[H];
#pragma unroll
    for (int f = 0; f < F; ++f) x[f] = sx[tl][f] = X[b * F + f];
    const float y = forward1(p, x, z1, z2);
    const float e = y - T[b];
    sl[tl] = e * e;
    const float dy = 2.f * e * inv_n;  // dL/dy with L = mean squared error
    sdy[tl] = dy;
    float d2[H];
#pragma unroll
    for (int u = 0; u < H; ++u) {
      sh2[tl][u] = z2[u] > 0.f ? z2[u] : 0.f;
      d2[u] = z2[u] > 0.f ? dy * p[OW3 + u] : 0.f;  // dL/dz2
      sd2[tl][u] = d2[u];
    }
#pragma unroll 4
    for (int q = 0; q < H; ++q) {
      float s = 0.f;
#pragma unroll
      for (int u = 0; u < H; ++u) s += p[OW2 + u * H + q] * d2[u];
      sd1[tl][q] = z1[q] > 0.f ? s : 0.f;  // dL/dz1
      sh1[tl][q] = z1[q] > 0.f ? z1[q] : 0.f;
    }
  }
  __syncthreads();
  float* out = part + int64_t(blockIdx.x) * kMlpParams;
  for (int q = threadIdx.x; q < kMlpParams; q += blockDim.x) {
    float s = 0.f;
    if (q < OB1) {  // W1[u][f] = sum_b d1[b][u] x[b][f]
      const int u = (q - OW1) / F, f = (q - OW1) % F;
      for (int i = 0; i < cnt; ++i) s += sd1[i][u] * sx[i][f];
    } else if (q < OW2) {
      for (int i = 0; i < cnt; ++i) s += sd1[i][q - OB1];
    } else if (q < OB2) {  // W2[u][v] = sum_b d2[b][u] h1[b][v]
      const int u = (q - OW2) / H, v = (q - OW2) % H;
      for (int i = 0; i < cnt; ++i) s += sd2[i][u] * sh1[i][v];
    } else if (q < OW3) {
      for (int i = 0; i < cnt; ++i) s += sd2[i][q - OB2];
    } else if (q < OB3) {
      for (int i = 0; i < cnt; ++i) s += sdy[i] * sh2[i][q - OW3];
    } else {
      for (int i = 0; i < cnt; ++i) s += sdy[i];
    }
    out[q] = s;
  }
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < cnt; ++i) s += sl[i];
    part_loss[blockIdx.x] = s;
  }
}

// grad[q] = sum over chunks of part[chunk][q] (chunk order); loss = sum part_loss * inv_n
__global__ __launch_bounds__(256) void mlp_grad_reduce(const float* __restrict__ part,
                                                       const float* __restrict__ part_loss,
                                                       int nchunks, float inv_n,
                                                       float* __restrict__ grad,
                                                       float* __restrict__ loss) {
  for (int q = threadIdx.x + blockIdx.x * blockDim.x; q < kMlpParams; q += blockDim.x * gridDim.x) {
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += part[int64_t(c) * kMlpParams + q];
    grad[q] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && loss) {
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += part_loss[c];
    *loss = s * inv_n;
  }
}

// Adam (Kingma & Ba): m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
// p <- p - lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
__global__ __launch_bounds__(256) void adam(float* __restrict__ p, const float* __restrict__ g,
                                            float* __restrict__ m, float* __restrict__ v, int64_t n,
                                            float lr, float b1, float b2, float eps, float c1,
                                            float c2) {
  for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < n;
       q += int64_t(gridDim.x) * blockDim.x) {
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.f - b1) * gq;
    const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
  }
}

}  // namespace

hipError_t launch_mlp_forward(const float* params, const float* X, int64_t n, float* Y,
                              const MlpNorm& norm, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(mlp_forward, dim3(uint32_t(blocks)), dim3(256), 0, s, params, X, n, Y, norm);
  return hipGetLastError();
}

hipError_t launch_mlp_normalize(float* X, float* T, int64_t n, const MlpNorm& norm, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(mlp_normalize, dim3(uint32_t(blocks)), dim3(256), 0, s, X, T, n, norm);
  return hipGetLastError();
}

int64_t mlp_partial_rows(int64_t n) { return (n + CHUNK - 1) / CHUNK; }

hipError_t launch_mlp_loss_grad(const float* params, const float* X, const float* T, int64_t n,
                                float* part, float* part_loss, float* grad, float* loss,
                                hipStream_t s) {
  if (n <= 0) return hipErrorInvalidValue;
  const int64_t chunks = mlp_partial_rows(n);
  const float inv_n = 1.f / float(n);
  hipLaunchKernelGGL(mlp_grad_partial, dim3(uint32_t(chunks)), dim3(CHUNK), 0, s, params, X, T, n,
                     inv_n, part, part_loss);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_grad_reduce, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, part,
                     part_loss, int(chunks), inv_n, grad, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, int64_t step,
                       float lr, float b1, float b2, float eps, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const float c1 = 1.f - powf(b1, float(step)), c2 = 1.f - powf(b2, float(step));
  hipLaunchKernelGGL(adam, dim3(uint32_t((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n, lr, b1,
                     b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace bsm
