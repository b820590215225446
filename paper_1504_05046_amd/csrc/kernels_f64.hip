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

// Fourth word of a raw (stride 0) buffer descriptor on gfx9-family targets: 32-bit data format,
// no swizzle; loads past num_records return 0.
constexpr int kRsrcWord3 = 0x00020000;
constexpr uint32_t kOutOfRange = 0x7FFFFFF8u;

template <int TM, int TN, int KC_, int NW_>
struct F64Cfg {
  static constexpr int KC = KC_;            // k-chunk staged per step
  static constexpr int NW = NW_;            // waves per workgroup
  static constexpr int NT = 64 * NW;        // threads per workgroup
  // LDS row strides (doubles), padded so that a half-wave's fragment reads hit distinct banks
  static constexpr int ASTR = KC == 16 ? KC + 1 : KC + 2;  // A chunk: TM rows x KC
  static constexpr int BSTR = TN + 16;                     // B chunk: KC rows x TN
  static constexpr int SLOTS = ((TM / 16) * (TN / 16) + NW - 1) / NW;  // 16x16 blocks per wave
  static constexpr int ARP = NT / KC;       // A rows staged per pass (KC threads per row)
  static constexpr int ALD = TM / ARP;      // A elements each thread stages per chunk
  static constexpr int BK = NT / TN;        // B k-rows staged per pass (TN threads per row)
  static constexpr int BLD = KC / BK;       // B elements each thread stages per chunk
  static_assert(KC % 16 == 0 && NT % KC == 0 && TM % ARP == 0, "A staging shape");
  static_assert(TN <= NT && NT % TN == 0 && KC % BK == 0, "B staging shape");
};

// The part of a task one wave runs when it owns NS of the sub-tile's 16x16 output blocks.
// Every wave of the workgroup walks the same k-chunks and meets the same barriers; NS is a
// compile-time constant so that the MFMA stream has no per-block branches.
template <int TM, int TN, int KC, int NW, int NS>
__device__ __forceinline__ void run_task(const Item& it, const Triple* __restrict__ tri,
                                         const ProductArgs& pa, int accumulate, int wave,
                                         double (*As)[TM * F64Cfg<TM, TN, KC, NW>::ASTR],
                                         double (*Bs)[F64Cfg<TM, TN, KC, NW>::KC * F64Cfg<TM, TN, KC, NW>::BSTR]) {
  using C = F64Cfg<TM, TN, KC, NW>;
  const int tid = threadIdx.x, lane = tid & 63;
  const int g = lane >> 4, i16 = lane & 15;
  const int h = it.h, w = it.w, ldc = it.ldc;
  const int bcn = (w + 15) >> 4;

  // this wave's output blocks q = wave, wave+4, ... (row-major over the sub-tile's 16x16 blocks)
  int a_u[NS > 0 ? NS : 1], b_u[NS > 0 ? NS : 1];
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    int q = wave + NW * j;
    int rb = q / bcn, cb = q - rb * bcn;
    a_u[j] = 16 * rb * C::ASTR;
    b_u[j] = 16 * cb;
  }
  d4 acc[NS > 0 ? NS : 1];
#pragma unroll
  for (int j = 0; j < NS; ++j) acc[j] = (d4){0.0, 0.0, 0.0, 0.0};

  // staging assignment: A chunk row-major (16 consecutive threads read one row's 16 k),
  // B chunk row-major (TN consecutive threads read one k-row's columns)
  const int ka = tid % KC, ra0 = tid / KC;
  const int cbl = tid % TN, kb0 = tid / TN;
  double ra[C::ALD], rb[C::BLD];

  // Staging loads go through buffer descriptors: a load whose offset lies past num_records
  // returns 0 instead of touching memory.  A's descriptor ends at row h of the sub-tile, so rows
  // beyond it read 0; the k-tail (k >= s_k would wrap into the next row) is sent out of range
  // explicitly.  B's descriptor ends at the last element of the sub-tile's columns, so k-rows
  // beyond s_k read 0; columns beyond w read finite neighbours that only feed output columns the
  // epilogue discards.
  auto load = [&](const Triple& t, int kk) {
    const int ks = tri_ks(t);
    const __amdgpu_buffer_rsrc_t ar = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double*>(pa.A + tri_a_off(t) + int64_t(it.r0) * ks), (short)0, h * ks * 8, kRsrcWord3);
    const __amdgpu_buffer_rsrc_t br = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double*>(pa.B + tri_b_off(t) + it.c0), (short)0, ((ks - 1) * ldc + w) * 8, kRsrcWord3);
    const bool kin = kk + ka < ks;
#pragma unroll
    for (int p = 0; p < C::ALD; ++p) {
      const uint32_t off = kin ? uint32_t(((ra0 + C::ARP * p) * ks + kk + ka) * 8) : kOutOfRange;
      ra[p] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(ar, off, 0, 0));
    }
#pragma unroll
    for (int p = 0; p < C::BLD; ++p) {
      const uint32_t off = uint32_t(((kk + kb0 + C::BK * p) * ldc + cbl) * 8);
      rb[p] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(br, off, 0, 0));
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int p = 0; p < C::ALD; ++p) As[buf][(ra0 + C::ARP * p) * C::ASTR + ka] = ra[p];
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
          // fragments are read in groups of up to 8 blocks to bound register use
#pragma unroll
          for (int j0 = 0; j0 < NS; j0 += 8) {
            constexpr int G = NS < 8 ? NS : 8;
            double av[G > 0 ? G : 1], bv[G > 0 ? G : 1];
#pragma unroll
            for (int j = 0; j < G; ++j) {
              if (j0 + j < NS) {
                av[j] = as[a_u[j0 + j] + 4 * s];
                bv[j] = bs[b_u[j0 + j] + 4 * s * C::BSTR];
              }
            }
#pragma unroll
            for (int j = 0; j < G; ++j)
              if (j0 + j < NS)
                acc[j0 + j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[j], bv[j], acc[j0 + j], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
          }
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
    int q = wave + NW * j;
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

template <int TM, int TN, int KC, int NW, int NS>
__device__ __forceinline__ void dispatch_ns(int ns, const Item& it, const Triple* __restrict__ tri,
                                            const ProductArgs& pa, int accumulate, int wave,
                                            double (*As)[TM * F64Cfg<TM, TN, KC, NW>::ASTR],
                                            double (*Bs)[F64Cfg<TM, TN, KC, NW>::KC * F64Cfg<TM, TN, KC, NW>::BSTR]) {
  if constexpr (NS > F64Cfg<TM, TN, KC, NW>::SLOTS) {
    return;
  } else {
    if (ns == NS) run_task<TM, TN, KC, NW, NS>(it, tri, pa, accumulate, wave, As, Bs);
    else dispatch_ns<TM, TN, KC, NW, NS + 1>(ns, it, tri, pa, accumulate, wave, As, Bs);
  }
}

template <int TM, int TN, int KC, int NW, int OCC>
__global__ __launch_bounds__(64 * NW, OCC) void f64_tiles(const Item* __restrict__ items,
                                                 const Triple* __restrict__ tri, XcdMap map,
                                                 const ProductArgs* __restrict__ prods,
                                                 ProductArgs single, int accumulate) {
  using C = F64Cfg<TM, TN, KC, NW>;
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
  const int ns = nb > wave ? (nb - wave + NW - 1) / NW : 0;  // output blocks of this wave
  dispatch_ns<TM, TN, KC, NW, 0>(ns, it, tri, pa, accumulate, wave, As, Bs);
}

#define BSM_F64_LAUNCH(ID, TM, TN, KC, NW, OCC)                                              \
  case ID:                                                                                   \
    hipLaunchKernelGGL((f64_tiles<TM, TN, KC, NW, OCC>), dim3(grid32), dim3(64 * NW), 0, stream, \
                       items, tri, map, prods, single, accumulate);                          \
    break;

hipError_t launch_f64(int variant, int64_t grid, const Item* items, const Triple* tri,
                      const XcdMap& map, const ProductArgs* prods, const ProductArgs& single,
                      int accumulate, hipStream_t stream) {
  if (grid <= 0) return hipSuccess;
  const uint32_t grid32 = static_cast<uint32_t>(grid);
  switch (variant) {
    BSM_F64_VARIANTS(BSM_F64_LAUNCH)
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace bsm
