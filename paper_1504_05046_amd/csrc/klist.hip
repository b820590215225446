// Device-built k-lists (S3 for products whose block triples would not fit a host list).
//
// One wave per C block (i, j): lane l holds words l, l + 64, ... of A's shape row i AND B's shape
// column j (the k with both A_ik and B_kj present); an exclusive prefix sum of the words' bit
// counts across the wave gives each lane the place of its first triple, so that the triples come
// out in ascending k, as the tile kernels expect.  A triple carries A_ik's and B_kj's offsets in
// the precision form's layout, the inner block size and k.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace bsm {

namespace {

__global__ __launch_bounds__(256) void fill_klists(const KJob* __restrict__ jobs, int64_t njobs,
                                                   const uint64_t* __restrict__ a_bits,
                                                   const uint64_t* __restrict__ bt_bits, int64_t wk,
                                                   const int64_t* __restrict__ a_tab,
                                                   const int64_t* __restrict__ bt_tab, int64_t K,
                                                   const int64_t* __restrict__ inner,
                                                   Triple* __restrict__ tri) {
  const int lane = threadIdx.x & 63;
  const int64_t q = int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (q >= njobs) return;  // the whole wave leaves together
  const KJob jb = jobs[q];
  const uint64_t* ar = a_bits + int64_t(jb.i) * wk;
  const uint64_t* br = bt_bits + int64_t(jb.j) * wk;
  const int64_t* at = a_tab + int64_t(jb.i) * K;
  const int64_t* bt = bt_tab + int64_t(jb.j) * K;
  uint32_t base = jb.tri_begin;
  const uint32_t end = jb.tri_begin + jb.count;  // writes never leave the job's range
  for (int64_t w0 = 0; w0 < wk; w0 += 64) {
    const int64_t w = w0 + lane;
    uint64_t x = w < wk ? (ar[w] & br[w]) : 0;
    const int c = __popcll(x);
    // inclusive prefix sum of c over the wave's lanes
    int incl = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int v = __shfl_up(incl, d, 64);
      if (lane >= d) incl += v;
    }
    const int total = __shfl(incl, 63, 64);
    uint32_t pos = base + uint32_t(incl - c);
    while (x) {
      const int64_t k = w * 64 + __ffsll(static_cast<unsigned long long>(x)) - 1;
      x &= x - 1;
      Triple t;
      t.a = uint64_t(at[k]) | (uint64_t(inner[k]) << 48);
      t.b = uint64_t(bt[k]) | (uint64_t(k) << 48);
      if (pos < end) tri[pos] = t;
      ++pos;
    }
    base += uint32_t(total);
  }
}

}  // namespace

hipError_t launch_fill_klists(const KJob* jobs, int64_t njobs, const DevKlists& d, Triple* tri,
                              hipStream_t stream) {
  if (njobs <= 0) return hipSuccess;
  const int64_t blocks = (njobs + 3) / 4;  // four waves per workgroup
  hipLaunchKernelGGL(fill_klists, dim3(uint32_t(blocks)), dim3(256), 0, stream, jobs, njobs,
                     d.a_bits, d.bt_bits, d.wk, d.a_tab, d.bt_tab, d.K, d.inner, tri);
  return hipGetLastError();
}

}  // namespace bsm
