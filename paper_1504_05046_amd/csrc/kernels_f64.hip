// FP64 tile contraction on gfx950 MFMA (v_mfma_f64_16x16x4_f64).
//
// One workgroup (4 waves) executes one task: a C sub-tile of h x w (h <= TM, w <= TN) and the
// whole k-list of its C block.  For every block triple of the list, in ascending k, the
// workgroup streams 16-wide k-chunks of A_ik (rows r0..r0+h) and B_kj (cols c0..c0+w) from HBM
// into LDS with coalesced 8-byte loads (double-buffered, one barrier per chunk), and the 4 waves
// share the sub-tile's 16x16 output blocks round-robin, each accumulating its blocks in FP64
// registers across the whole k-list.  The epilogue writes alpha*acc (+C) once per element: the
// paper's multiply task and reduction task fused, with no temporaries (Sec. 3.2, Fig. 3).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace bsm {

typedef double d4 __attribute__((ext_vector_type(4)));

template <int TM, int TN, int KC_>
struct F64Cfg {
  static constexpr int KC = KC_;            // k-chunk staged per step
  static constexpr int ASTR = KC + 1;       // LDS row stride of the A chunk (rows x KC)
  static constexpr int BSTR = TN + 16;      // LDS row stride of the B chunk (KC x cols)
  static constexpr int SLOTS = (TM / 16) * (TN / 16) / 4;  // 16x16 output blocks per wave
  static constexpr int ALD = TM / 16;       // A elements each thread stages per chunk
  static constexpr int BK = 256 / TN;       // B rows covered by one pass of 256 threads
  static constexpr int BLD = KC / BK;       // B elements each thread stages per chunk
  static_assert(TN <= 256 && 256 % TN == 0 && KC % BK == 0, "tile shape");
  static_assert(SLOTS >= 1, "tile too small for 4 waves");
};

// The part of a task one wave runs when it owns NS of the sub-tile's 16x16 output blocks.
// Every wave of the workgroup walks the same k-chunks and meets the same barriers; NS is a
// compile-time constant so that the MFMA stream has no per-block branches.
template <int TM, int TN, int KC, int NS>
__device__ __forceinline__ void run_task(const Item& it, const Triple* __restrict__ tri,
                                         const ProductArgs& pa, int accumulate, int wave,
                                         double (*As)[TM * F64Cfg<TM, TN, KC>::ASTR],
                                         double (*Bs)[F64Cfg<TM, TN, KC>::KC * F64Cfg<TM, TN, KC>::BSTR]) {
  using C = F64Cfg<TM, TN, KC>;
  const int tid = threadIdx.x, lane = tid & 63;
  const int g = lane >> 4, i16 = lane & 15;
  const int h = it.h, w = it.w, ldc = it.ldc;
  const int bcn = (w + 15) >> 4;

  // this wave's output blocks q = wave, wave+4, ... (row-major over the sub-tile's 16x16 blocks)
  int a_u[NS > 0 ? NS : 1], b_u[NS > 0 ? NS : 1];
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    int q = wave + 4 * j;
    int rb = q / bcn, cb = q - rb * bcn;
    a_u[j] = 16 * rb * C::ASTR;
    b_u[j] = 16 * cb;
  }
  d4 acc[NS > 0 ? NS : 1];
#pragma unroll
  for (int j = 0; j < NS; ++j) acc[j] = (d4){0.0, 0.0, 0.0, 0.0};

  // staging assignment: A chunk row-major (16 consecutive threads read one row's 16 k),
  // B chunk row-major (TN consecutive threads read one k-row's columns)
  const int ka = tid & 15, ra0 = tid >> 4;
  const int cbl = tid % TN, kb0 = tid / TN;
  double ra[C::ALD], rb[C::BLD];

  auto load = [&](const Triple& t, int kk) {
    const int ks = tri_ks(t);
    const double* Ab = pa.A + tri_a_off(t) + int64_t(it.r0) * ks + kk;
    const double* Bb = pa.B + tri_b_off(t) + int64_t(kk) * ldc + it.c0;
    const bool kin = kk + ka < ks;
#pragma unroll
    for (int p = 0; p < C::ALD; ++p) {
      int row = ra0 + 16 * p;
      ra[p] = (kin && row < h) ? Ab[int64_t(row) * ks + ka] : 0.0;
    }
#pragma unroll
    for (int p = 0; p < C::BLD; ++p) {
      int kr = kb0 + C::BK * p;
      rb[p] = (cbl < w && kk + kr < ks) ? Bb[int64_t(kr) * ldc + cbl] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int p = 0; p < C::ALD; ++p) As[buf][(ra0 + 16 * p) * C::ASTR + ka] = ra[p];
#pragma unroll
    for (int p = 0; p < C::BLD; ++p) Bs[buf][(kb0 + C::BK * p) * C::BSTR + cbl] = rb[p];
  };

  const uint32_t te = it.tri_begin + it.tri_count;
  uint32_t t = it.tri_begin;
  int kk = 0;
  Triple tc;
  if (t < te) {
    tc = tri[t];
    load(tc, 0);
    store(0);
  }
  __syncthreads();
  int buf = 0;
  while (t < te) {
    const int ks = tri_ks(tc);
    const int nsteps = (min(C::KC, ks - kk) + 3) >> 2;  // 4-deep MFMA steps holding data
    // next chunk: the rest of this block, else the next triple
    uint32_t tn = t;
    int kn = kk + C::KC;
    Triple tnx = tc;
    if (kn >= ks) {
      tn = t + 1;
      kn = 0;
      if (tn < te) tnx = tri[tn];
    }
    const bool more = tn < te;
    if (more) load(tnx, kn);

    if (NS > 0) {
      const double* as = As[buf] + i16 * C::ASTR + g;
      const double* bs = Bs[buf] + g * C::BSTR + i16;
      // one 4-deep MFMA step per iteration; steps past the block's end hold only zeros and are
      // skipped (the condition is the same for the whole wave)
#pragma unroll
      for (int s = 0; s < C::KC / 4; ++s) {
        if (s < nsteps) {
          double av[NS > 0 ? NS : 1], bv[NS > 0 ? NS : 1];
#pragma unroll
          for (int j = 0; j < NS; ++j) {
            av[j] = as[a_u[j] + 4 * s];
            bv[j] = bs[b_u[j] + 4 * s * C::BSTR];
          }
#pragma unroll
          for (int j = 0; j < NS; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[j], bv[j], acc[j], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
    t = tn;
    kk = kn;
    tc = tnx;
  }

  // epilogue: on gfx950 the FP64 16x16x4 result puts row g + 4r (r = 0..3), column i16 of a
  // 16x16 block in register r of lane 16g + i16
  double* Cb = pa.C + it.c_off + int64_t(it.r0) * ldc + it.c0;
  const double alpha = pa.alpha;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    int q = wave + 4 * j;
    int rbk = q / bcn, cbk = q - rbk * bcn;
    int col = 16 * cbk + i16;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int row = 16 * rbk + g + 4 * r;
      if (row < h && col < w) {
        double* pc = Cb + int64_t(row) * ldc + col;
        double v = alpha * acc[j][r];
        *pc = accumulate ? v + *pc : v;
      }
    }
  }
}

template <int TM, int TN, int KC, int NS>
__device__ __forceinline__ void dispatch_ns(int ns, const Item& it, const Triple* __restrict__ tri,
                                            const ProductArgs& pa, int accumulate, int wave,
                                            double (*As)[TM * F64Cfg<TM, TN, KC>::ASTR],
                                            double (*Bs)[F64Cfg<TM, TN, KC>::KC * F64Cfg<TM, TN, KC>::BSTR]) {
  if constexpr (NS > F64Cfg<TM, TN, KC>::SLOTS) {
    return;
  } else {
    if (ns == NS) run_task<TM, TN, KC, NS>(it, tri, pa, accumulate, wave, As, Bs);
    else dispatch_ns<TM, TN, KC, NS + 1>(ns, it, tri, pa, accumulate, wave, As, Bs);
  }
}

template <int TM, int TN, int KC, int OCC>
__global__ __launch_bounds__(256, OCC) void f64_tiles(const Item* __restrict__ items,
                                                 const Triple* __restrict__ tri, XcdMap map,
                                                 const ProductArgs* __restrict__ prods,
                                                 ProductArgs single, int accumulate) {
  using C = F64Cfg<TM, TN, KC>;
  __shared__ double As[2][TM * C::ASTR];
  __shared__ double Bs[2][C::KC * C::BSTR];

  // XCD-aware task lookup: the hardware deals workgroups round-robin over the 8 XCDs, so
  // workgroup 8q + x runs on XCD x and takes that XCD's q-th task.
  const int x = blockIdx.x % kXcds, qx = blockIdx.x / kXcds;
  const int idx = map.begin[x] + qx;
  if (idx >= map.begin[x + 1]) return;
  const Item it = items[idx];
  const ProductArgs pa = prods ? prods[it.product] : single;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nb = ((it.h + 15) >> 4) * ((it.w + 15) >> 4);
  const int ns = nb > wave ? (nb - wave + 3) >> 2 : 0;  // output blocks of this wave
  dispatch_ns<TM, TN, KC, 0>(ns, it, tri, pa, accumulate, wave, As, Bs);
}

#define BSM_F64_VARIANT(ID, TM, TN, KC, OCC)                                                 \
  case ID:                                                                                   \
    hipLaunchKernelGGL((f64_tiles<TM, TN, KC, OCC>), g, b, 0, stream, items, tri, map, prods, \
                       single, accumulate);                                                  \
    break;

hipError_t launch_f64(int variant, int64_t grid, const Item* items, const Triple* tri,
                      const XcdMap& map, const ProductArgs* prods, const ProductArgs& single,
                      int accumulate, hipStream_t stream) {
  if (grid <= 0) return hipSuccess;
  dim3 g(static_cast<uint32_t>(grid)), b(256);
  switch (variant) {
    BSM_F64_VARIANT(0, 128, 128, 16, 2)
    BSM_F64_VARIANT(1, 64, 64, 16, 1)
    BSM_F64_VARIANT(2, 32, 32, 16, 1)
    BSM_F64_VARIANT(3, 128, 128, 32, 1)
    BSM_F64_VARIANT(4, 128, 128, 16, 1)
    BSM_F64_VARIANT(5, 64, 64, 32, 1)
    BSM_F64_VARIANT(6, 128, 64, 16, 2)
    BSM_F64_VARIANT(7, 64, 64, 16, 3)
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace bsm
