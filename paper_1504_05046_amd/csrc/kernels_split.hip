// Operand preparation passes (HBM-bound, ahead of the tile kernels): conversion for the
// reduced-precision forms (FP32: the packed layout is kept, only the element type changes;
// split-bf16: three slice planes in 32-wide k-panels, transposing on the way where needed), the
// transposition of an operand that the product reads as X^T (Sec. 2.1's transposed variants) into
// the product's packed layout, the real embedding of complex operands and the complex epilogue,
// and the copies, permutations and reductions of the low-rank, contraction and k_split paths.
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

// Round to the nearest value with 8 significant bits (bf16 precision), ties to even, by adding
// half an ulp of the 8-bit grid to the bit pattern.  Exact for finite values in FP32's normal
// range; non-finite values are passed through.
__device__ inline double round8(double a) {
  uint64_t b = uint64_t(__double_as_longlong(a));
  if (((b >> 52) & 0x7FF) == 0x7FF) return a;
  b += ((uint64_t(1) << 44) - 1) + ((b >> 45) & 1);
  b &= ~((uint64_t(1) << 45) - 1);
  return __longlong_as_double(int64_t(b));
}

// Bits of a value that already has at most 8 significant bits, as bf16.
__device__ inline uint16_t bf16_bits(double x) {
  return uint16_t(__float_as_uint(float(x)) >> 16);
}

// a = a0 + a1 + a2 + (error below 2^-24 |a|): each slice is the residual rounded to 8 bits;
// the residuals a - a0 and (a - a0) - a1 are exact in FP64.
__device__ inline void split3(double a, uint16_t& s0, uint16_t& s1, uint16_t& s2) {
  const double a0 = round8(a);
  const double r1 = a - a0;
  const double a1 = round8(r1);
  const double a2 = round8(r1 - a1);
  s0 = bf16_bits(a0);
  s1 = bf16_bits(a1);
  s2 = bf16_bits(a2);
}

static_assert(kSliceK == 32, "panel indexing below assumes 32-wide k-panels");

// Four consecutive slice values of one plane as one 8-byte word (the lowest k first).
__device__ inline uint64_t pack4(const uint16_t (&x)[4]) {
  return uint64_t(x[0]) | (uint64_t(x[1]) << 16) | (uint64_t(x[2]) << 32) | (uint64_t(x[3]) << 48);
}

// Splits four values and stores the three slices' four bf16 each at element offset o (a multiple
// of 4, so every store is one aligned 8-byte word).
__device__ inline void split_store4(const double (&v)[4], uint16_t* d0, uint16_t* d1, uint16_t* d2,
                                    int64_t o) {
  uint16_t x0[4], x1[4], x2[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) split3(v[j], x0[j], x1[j], x2[j]);
  *reinterpret_cast<uint64_t*>(d0 + o) = pack4(x0);
  *reinterpret_cast<uint64_t*>(d1 + o) = pack4(x1);
  *reinterpret_cast<uint64_t*>(d2 + o) = pack4(x2);
}

// One workgroup per table entry: an operand block, or a piece of one (the planner gives every
// 32-wide k-panel its own entry), written as three slices into the planes (plane p at
// dst + p * plane) with the inner size padded with zeros to a multiple of 32, in 32-wide k-panels
// (element (r, k) of a block of R rows at (k / 32) * 32 R + 32 r + k % 32).  Each thread handles
// four consecutive k of one row (one 8-byte store per plane; entry offsets in the planes are
// multiples of 32 elements).  B blocks are transposed through LDS in 32 x 64 tiles so that both
// the reads and the writes are coalesced.
__global__ __launch_bounds__(256) void split_bf16x3(const SplitBlock* __restrict__ blocks,
                                                    const double* __restrict__ src,
                                                    uint16_t* __restrict__ dst, int64_t plane) {
  __shared__ double tile[32][65];
  const SplitBlock b = blocks[blockIdx.x];
  const int ks32 = int(pad_k(b.ks));
  const double* sb = src + b.src_off;
  uint16_t* d0 = dst + b.dst_off;
  uint16_t* d1 = d0 + plane;
  uint16_t* d2 = d1 + plane;
  if (!b.transpose) {
    // quad u: panel u / (8 rows), row (u mod 8 rows) / 8, k-quad u mod 8 of the panel; the
    // destination of a quad is 4 u (panels are consecutive, rows 32 elements apart in a panel)
    const int quads = b.rows * (ks32 >> 2);
    for (int u = threadIdx.x; u < quads; u += blockDim.x) {
      const int pr = u / (b.rows * 8), e = u - pr * (b.rows * 8);
      const int r = e >> 3, k = pr * kSliceK + ((e & 7) << 2);
      const double* row = sb + int64_t(r) * b.ld_src;
      double v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = k + j < b.ks ? row[k + j] : 0.0;
      split_store4(v, d0, d1, d2, int64_t(u) << 2);
    }
    return;
  }
  // source: ks rows x `rows` columns (ld = ld_src); destination: `rows` x ks32
  for (int c0 = 0; c0 < b.rows; c0 += 64) {
    for (int k0 = 0; k0 < ks32; k0 += 32) {
      for (int e = threadIdx.x; e < 32 * 64; e += blockDim.x) {
        const int kk = e >> 6, cc = e & 63;
        const int k = k0 + kk, c = c0 + cc;
        tile[kk][cc] = (k < b.ks && c < b.rows) ? sb[int64_t(k) * b.ld_src + c] : 0.0;
      }
      __syncthreads();
      // 64 columns x 8 k-quads: thread f takes column f / 8, quad f mod 8
      for (int f = threadIdx.x; f < 64 * 8; f += blockDim.x) {
        const int cc = f >> 3, q = (f & 7) << 2;
        const int c = c0 + cc;
        if (c < b.rows) {
          double v[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) v[j] = tile[q + j][cc];
          split_store4(v, d0, d1, d2, int64_t(k0) * b.rows + int64_t(c) * kSliceK + q);
        }
      }
      __syncthreads();
    }
  }
}

// One workgroup per piece (at most 64 source rows): the piece goes through LDS in 64 x 64 tiles
// (reads coalesced along the source rows, writes along the destination rows), rounded to T.  The
// 65-element row pitch spreads both phases over the LDS banks.
template <typename T>
__global__ __launch_bounds__(256) void transpose_blocks(const XposeBlock* __restrict__ blocks,
                                                        const double* __restrict__ src,
                                                        T* __restrict__ dst) {
  __shared__ double tile[64][65];
  const XposeBlock b = blocks[blockIdx.x];
  const double* sb = src + b.src_off;
  T* db = dst + b.dst_off;
  for (int r0 = 0; r0 < b.rows; r0 += 64)
    for (int c0 = 0; c0 < b.cols; c0 += 64) {
      const int th = b.rows - r0 < 64 ? b.rows - r0 : 64;
      const int tw = b.cols - c0 < 64 ? b.cols - c0 : 64;
      for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
        const int rr = e >> 6, cc = e & 63;
        if (rr < th && cc < tw) tile[rr][cc] = sb[int64_t(r0 + rr) * b.ld_src + c0 + cc];
      }
      __syncthreads();
      for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
        const int cc = e >> 6, rr = e & 63;
        if (rr < th && cc < tw) db[int64_t(c0 + cc) * b.ld_dst + r0 + rr] = T(tile[rr][cc]);
      }
      __syncthreads();
    }
}

template <typename T>
static hipError_t launch_transpose(const XposeBlock* blocks, int64_t nblocks, const double* src,
                                   T* dst, hipStream_t stream) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(transpose_blocks<T>, dim3(uint32_t(nblocks)), dim3(256), 0, stream, blocks,
                     src, dst);
  return hipGetLastError();
}

hipError_t launch_transpose_f64(const XposeBlock* blocks, int64_t nblocks, const double* src,
                                double* dst, hipStream_t stream) {
  return launch_transpose(blocks, nblocks, src, dst, stream);
}

hipError_t launch_transpose_f32(const XposeBlock* blocks, int64_t nblocks, const double* src,
                                float* dst, hipStream_t stream) {
  return launch_transpose(blocks, nblocks, src, dst, stream);
}

// One workgroup per piece (up to kZBand rows of a complex block): op(X) goes through LDS in
// 32 x 32 tiles of complex elements (reads along the stored rows, transposed or not; writes along
// the embedded rows) and is written as [[Re, -Im], [Im, Re]] (left operand, row pitch 2 cols) or
// [Re; Im] (right operand); the imaginary half starts full_rows rows below the real one.
__global__ __launch_bounds__(256) void embed_complex(const ZBlock* __restrict__ blocks,
                                                     const double2* __restrict__ src,
                                                     double* __restrict__ dst) {
  __shared__ double2 tile[32][33];
  const ZBlock b = blocks[blockIdx.x];
  const bool tr = (b.mode & kZTrans) != 0, cj = (b.mode & kZConj) != 0;
  const bool right = (b.mode & kZRight) != 0;
  const double2* sb = src + b.src_off;
  double* db = dst + b.dst_off;
  const int R = b.rows, W = b.cols, RF = b.full_rows;
  for (int x0 = 0; x0 < R; x0 += 32)
    for (int y0 = 0; y0 < W; y0 += 32) {
      for (int e = threadIdx.x; e < 32 * 32; e += blockDim.x) {
        const int xx = tr ? (e & 31) : (e >> 5), yy = tr ? (e >> 5) : (e & 31);
        if (x0 + xx < R && y0 + yy < W) {
          const int64_t idx = tr ? int64_t(y0 + yy) * RF + x0 + xx : int64_t(x0 + xx) * W + y0 + yy;
          double2 v = sb[idx];
          if (cj) v.y = -v.y;
          tile[xx][yy] = v;
        }
      }
      __syncthreads();
      for (int e = threadIdx.x; e < 32 * 32; e += blockDim.x) {
        const int xx = e >> 5, yy = e & 31, x = x0 + xx, y = y0 + yy;
        if (x < R && y < W) {
          const double2 v = tile[xx][yy];
          if (right) {
            db[int64_t(x) * W + y] = v.x;
            db[int64_t(RF + x) * W + y] = v.y;
          } else {
            const int64_t ld = 2 * int64_t(W);
            db[int64_t(x) * ld + y] = v.x;
            db[int64_t(x) * ld + W + y] = -v.y;
            db[int64_t(RF + x) * ld + y] = v.y;
            db[int64_t(RF + x) * ld + W + y] = v.x;
          }
        }
      }
      __syncthreads();
    }
}

hipError_t launch_embed_complex(const ZBlock* blocks, int64_t nblocks, const double* src,
                                double* dst, hipStream_t stream) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(embed_complex, dim3(uint32_t(nblocks)), dim3(256), 0, stream, blocks,
                     reinterpret_cast<const double2*>(src), dst);
  return hipGetLastError();
}

// One workgroup per piece of a complex C block: C = alpha (Re + i Im) (+ C) from the real
// product's [Re; Im] block, stored interleaved as complex FP64 (V = double2) or complex FP32
// (float2), for the piece's elements [e0, e1).
template <typename V>
__global__ __launch_bounds__(256) void complex_epilogue(const ZCBlock* __restrict__ blocks,
                                                        const double* __restrict__ P,
                                                        V* __restrict__ C, double ar, double ai,
                                                        int accumulate) {
  const ZCBlock b = blocks[blockIdx.x];
  const double* pr = P + 2 * b.off;
  const double* pi = pr + b.n;
  V* c = C + b.off;
  for (int64_t e = b.e0 + threadIdx.x; e < b.e1; e += blockDim.x) {
    const double xr = pr[e], xi = pi[e];
    double vr = ar * xr - ai * xi, vi = ar * xi + ai * xr;
    if (accumulate) {
      const V old = c[e];
      vr += double(old.x);
      vi += double(old.y);
    }
    V out;
    out.x = decltype(out.x)(vr);
    out.y = decltype(out.y)(vi);
    c[e] = out;
  }
}

hipError_t launch_complex_epilogue(const ZCBlock* blocks, int64_t nblocks, const double* P,
                                   void* C, int c_f32, double ar, double ai, int accumulate,
                                   hipStream_t stream) {
  if (nblocks <= 0) return hipSuccess;
  if (c_f32)
    hipLaunchKernelGGL(complex_epilogue<float2>, dim3(uint32_t(nblocks)), dim3(256), 0, stream,
                       blocks, P, static_cast<float2*>(C), ar, ai, accumulate);
  else
    hipLaunchKernelGGL(complex_epilogue<double2>, dim3(uint32_t(nblocks)), dim3(256), 0, stream,
                       blocks, P, static_cast<double2*>(C), ar, ai, accumulate);
  return hipGetLastError();
}

// One workgroup per tensor block: reads follow the source block (coalesced), each element's
// destination is the mixed-radix decomposition of its index against the block's extents, weighted
// by the destination strides.
template <typename T>
__global__ __launch_bounds__(256) void permute_blocks(const PermBlock* __restrict__ blocks,
                                                      const double* __restrict__ src,
                                                      T* __restrict__ dst, int accumulate) {
  const PermBlock b = blocks[blockIdx.x];
  const double* s = src + b.src_off;
  T* d = dst + b.dst_off;
  // a piece holds fewer than 2^32 elements of one block: 32-bit index arithmetic
  for (int64_t e = b.e0 + threadIdx.x; e < b.e1; e += blockDim.x) {
    uint32_t rem = uint32_t(e);
    int64_t o = 0;
    for (int m = b.order - 1; m >= 0; --m) {
      const uint32_t ext = uint32_t(b.ext[m]);
      const uint32_t q = rem / ext;
      o += int64_t(rem - q * ext) * b.dst_stride[m];
      rem = q;
    }
    const double v = s[e];
    d[o] = T(accumulate ? v + double(d[o]) : v);
  }
}

hipError_t launch_permute_blocks(const PermBlock* blocks, int64_t nblocks, const double* src,
                                 void* dst, int c_f32, int accumulate, hipStream_t stream) {
  if (nblocks <= 0) return hipSuccess;
  if (c_f32)
    hipLaunchKernelGGL(permute_blocks<float>, dim3(uint32_t(nblocks)), dim3(256), 0, stream,
                       blocks, src, static_cast<float*>(dst), accumulate);
  else
    hipLaunchKernelGGL(permute_blocks<double>, dim3(uint32_t(nblocks)), dim3(256), 0, stream,
                       blocks, src, static_cast<double*>(dst), accumulate);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void fill_zero(double* __restrict__ d, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += stride) d[e] = 0.0;
}

template <typename T>
__global__ __launch_bounds__(256) void reduce_splits(const double* __restrict__ P, int S,
                                                     int64_t n, T* __restrict__ C, double alpha,
                                                     int accumulate) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += stride) {
    double acc = P[e];
    for (int s = 1; s < S; ++s) acc += P[int64_t(s) * n + e];
    const double v = alpha * acc;
    C[e] = T(accumulate ? v + double(C[e]) : v);
  }
}

static int64_t flat_grid(int64_t n) {
  int64_t blocks = (n + 255) / 256;
  return blocks < 1 ? 1 : (blocks > 256 * 32 ? 256 * 32 : blocks);
}

hipError_t launch_fill_zero(double* dst, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero, dim3(uint32_t(flat_grid(n))), dim3(256), 0, stream, dst, n);
  return hipGetLastError();
}

hipError_t launch_reduce_splits(const double* P, int S, int64_t n, void* C, int c_f32,
                                double alpha, int accumulate, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const dim3 grid(uint32_t(flat_grid(n)));
  if (c_f32)
    hipLaunchKernelGGL(reduce_splits<float>, grid, dim3(256), 0, stream, P, S, n,
                       static_cast<float*>(C), alpha, accumulate);
  else
    hipLaunchKernelGGL(reduce_splits<double>, grid, dim3(256), 0, stream, P, S, n,
                       static_cast<double*>(C), alpha, accumulate);
  return hipGetLastError();
}

// One workgroup per run; 16-byte accesses when both ends are 16-byte aligned, else 8-byte ones.
__global__ __launch_bounds__(256) void copy_blocks(const CopyBlock* __restrict__ blocks,
                                                   const double* __restrict__ src,
                                                   double* __restrict__ dst) {
  const CopyBlock b = blocks[blockIdx.x];
  const double* s = src + b.src_off;
  double* d = dst + b.dst_off;
  if (((reinterpret_cast<uintptr_t>(s) | reinterpret_cast<uintptr_t>(d)) & 15) == 0) {
    const int64_t n2 = b.n / 2;
    const double2* s2 = reinterpret_cast<const double2*>(s);
    double2* d2 = reinterpret_cast<double2*>(d);
    for (int64_t e = threadIdx.x; e < n2; e += blockDim.x) d2[e] = s2[e];
    if ((b.n & 1) && threadIdx.x == 0) d[b.n - 1] = s[b.n - 1];
  } else {
    for (int64_t e = threadIdx.x; e < b.n; e += blockDim.x) d[e] = s[e];
  }
}

hipError_t launch_copy_blocks(const CopyBlock* blocks, int64_t nblocks, const double* src,
                              double* dst, hipStream_t stream) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_blocks, dim3(uint32_t(nblocks)), dim3(256), 0, stream, blocks, src, dst);
  return hipGetLastError();
}

hipError_t launch_split_bf16x3(const SplitBlock* blocks, int64_t nblocks, const double* src,
                               uint16_t* dst, int64_t plane, hipStream_t stream) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(split_bf16x3, dim3(uint32_t(nblocks)), dim3(256), 0, stream, blocks, src, dst,
                     plane);
  return hipGetLastError();
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
