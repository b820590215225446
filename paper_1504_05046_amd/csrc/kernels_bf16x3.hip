// Split-bf16 tile contraction on gfx950 (v_mfma_f32_16x16x32_bf16).
//
// Each FP64 operand element is held as three bf16 slices a = a0 + a1 + a2 (written by the split
// pass).  A block product is formed from the six slice products of order <= 2,
//   a2 b0 + a1 b1 + a0 b2 + a1 b0 + a0 b1 + a0 b0,
// accumulated in FP32 inside one block product A_ik B_kj and added into FP64 registers when the
// triple ends; the epilogue writes alpha*sum (+C) in FP64 once per element.
//
// One workgroup of 8 waves runs one task (a C sub-tile of up to 128 x 128 and its k-list).  The
// k-list is streamed in 32-deep chunks (one MFMA step, one k-panel of the slice planes, whose rows
// are contiguous): the three slices of A (rows) and of B (columns, stored k-contiguous) go through
// double-buffered LDS with 16-byte loads and stores.
// Each wave owns one rectangle of the sub-tile's 16x16 output blocks, from the same balanced table
// as the FP64/FP32 kernel (the busiest wave owns the fewest blocks any rectangle tiling allows), and
// reuses every fragment it reads from LDS across a row or column of its blocks.
//
// LDS layout: one 64-byte row (32 bf16 of a k-panel) per A row or B column, no padding; the
// 16-byte granule o of row r sits at granule o ^ ((r >> 1) & 3).  Measured on gfx950 with the LDS
// bank-conflict counter, this makes both the fragment reads (16 rows x 4 granules per ds_read_b128)
// and the staging stores (4 lanes per row per ds_write_b128) conflict-free, where plain 64-byte or
// 80-byte rows conflict on one of the two.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "uniform.hpp"
#include "wave_rects.inc"

namespace bsm {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kRsrcWord3b = 0x00020000;

__device__ inline uint32_t lower_bound_k3(const Triple* __restrict__ tri, uint32_t tb, uint32_t te,
                                          int k) {
  while (tb < te) {
    uint32_t mid = tb + ((te - tb) >> 1);
    if (tri_k(tri[mid]) < k) tb = mid + 1;
    else te = mid;
  }
  return tb;
}

template <int TM, int TN, int NW>
struct B3Cfg {
  static constexpr int KC = kSliceK;           // one MFMA step per chunk
  static constexpr int NT = 64 * NW;
  static constexpr int RS = KC;                // LDS row: 32 bf16 = 64 bytes
  static constexpr int ASZ = 3 * TM * RS;      // bf16 elements of one A stage (3 slices)
  static constexpr int BSZ = 3 * TN * RS;
  static constexpr int AG = 3 * TM * (KC / 8); // 16-byte granules of one A stage
  static constexpr int BG = 3 * TN * (KC / 8);
  static constexpr int ALD = AG / NT, BLD = BG / NT;
  static_assert(AG % NT == 0 && BG % NT == 0, "bf16 tile shape");
  // bf16 offset of granule o (8 bf16) of LDS row r
  __device__ static inline int gpos(int r, int o) { return r * RS + ((o ^ ((r >> 1) & 3)) << 3); }
};

template <int TM, int TN, int NW, bool RESUME, int NR, int NC>
__device__ __forceinline__ void run_b3(const TileArgs& a, const Item& it, const ProductArgs& pa,
                                       int rb0, int cb0, uint16_t* As, uint16_t* Bs) {
  using C = B3Cfg<TM, TN, NW>;
  constexpr int NRA = NR > 0 ? NR : 1, NCA = NC > 0 ? NC : 1;
  const int tid = threadIdx.x, lane = tid & 63;
  const int g = lane >> 4, i16 = lane & 15;
  const int h = it.h, w = it.w, ldc = it.ldc;
  const int64_t c_base = it.c_off + int64_t(it.r0) * ldc + it.c0;

  d4 acc[NRA][NCA];
  f4 acc32[NRA][NCA];
  const __amdgpu_buffer_rsrc_t prs = __builtin_amdgcn_make_buffer_rsrc(
      uni_ptr(pa.P + c_base), (short)0, uni(RESUME ? ((h - 1) * ldc + w) * 8 : 0), kRsrcWord3b);
#pragma unroll
  for (int x = 0; x < NR; ++x)
#pragma unroll
    for (int y = 0; y < NC; ++y) {
      acc[x][y] = (d4){0.0, 0.0, 0.0, 0.0};
      acc32[x][y] = (f4){0.f, 0.f, 0.f, 0.f};
      if constexpr (RESUME) {
        const int col = 16 * (cb0 + y) + i16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * (rb0 + x) + 4 * g + r;
          const uint32_t off = (row < h && col < w) ? uint32_t((row * ldc + col) * 8) : 0x7FFFFFF0u;
          acc[x][y][r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(prs, off, 0, 0));
        }
      }
    }

  const uint16_t* Ag = static_cast<const uint16_t*>(pa.A);
  const uint16_t* Bg = static_cast<const uint16_t*>(pa.B);
  // Two sets of staging registers: while chunk c is computed from LDS, the loads of chunk c + 2
  // are in flight into one set and chunk c + 1 waits in the other for its turn in LDS.
  struct Regs {
    u4 a[C::ALD], b[C::BLD];
  };
  Regs R0, R1;
  // granule q of a stage: slice q / (rows*4), row (q % (rows*4)) / 4, k-octet q % 4.  The chunk
  // is one 32-wide k-panel of the slice planes, whose rows are contiguous: the sub-tile's rows
  // r0..r0+h of A_ik (a panel of ldm rows) and columns c0..c0+w of B_kj (a panel of ldc columns)
  // are one run of 64-byte rows each.  A chunk past the end of the k-list is loaded through empty
  // descriptors (zeros, no memory access), so that every chunk issues the same loads.
  auto load = [&](const Triple& t, int kk, bool valid, Regs& R) {
    const uint16_t* ab = Ag + tri_a_off(t) + int64_t(kk) * it.ldm + int64_t(it.r0) * kSliceK;
    const uint16_t* bb = Bg + tri_b_off(t) + int64_t(kk) * it.ldc + int64_t(it.c0) * kSliceK;
    // rows past h (columns past w) fall outside the descriptor and read 0
    const int na = uni(valid ? h * kSliceK * 2 : 0), nb = uni(valid ? w * kSliceK * 2 : 0);
#pragma unroll
    for (int p = 0; p < C::ALD; ++p) {
      const int q = tid + C::NT * p;
      const int s = q / (TM * 4), rem = q - s * (TM * 4);
      const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
          uni_ptr(const_cast<uint16_t*>(ab + s * pa.a_plane)), (short)0, na, kRsrcWord3b);
      R.a[p] = __builtin_amdgcn_raw_buffer_load_b128(r, uint32_t(((rem >> 2) * kSliceK + 8 * (rem & 3)) * 2), 0, 0);
    }
#pragma unroll
    for (int p = 0; p < C::BLD; ++p) {
      const int q = tid + C::NT * p;
      const int s = q / (TN * 4), rem = q - s * (TN * 4);
      const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
          uni_ptr(const_cast<uint16_t*>(bb + s * pa.b_plane)), (short)0, nb, kRsrcWord3b);
      R.b[p] = __builtin_amdgcn_raw_buffer_load_b128(r, uint32_t(((rem >> 2) * kSliceK + 8 * (rem & 3)) * 2), 0, 0);
    }
  };
  auto store = [&](const Regs& R, int buf) {
#pragma unroll
    for (int p = 0; p < C::ALD; ++p) {
      const int q = tid + C::NT * p;
      const int s = q / (TM * 4), rem = q - s * (TM * 4);
      *reinterpret_cast<u4*>(As + buf * C::ASZ + s * TM * C::RS + C::gpos(rem >> 2, rem & 3)) = R.a[p];
    }
#pragma unroll
    for (int p = 0; p < C::BLD; ++p) {
      const int q = tid + C::NT * p;
      const int s = q / (TN * 4), rem = q - s * (TN * 4);
      *reinterpret_cast<u4*>(Bs + buf * C::BSZ + s * TN * C::RS + C::gpos(rem >> 2, rem & 3)) = R.b[p];
    }
  };

  // A chunk's place in the k-list: triple index t (valid while t < te), its triple, and the
  // offset kk of the chunk within the block's padded inner dimension.
  struct Pos {
    uint32_t t;
    int kk;
    Triple tri;
  };
  uint32_t te = it.tri_begin + it.tri_count;
  uint32_t t0 = it.tri_begin;
  if (a.k_lo > 0) t0 = uni(lower_bound_k3(a.tri, t0, te, a.k_lo));
  if (a.k_hi < kNoKLimit) te = uni(lower_bound_k3(a.tri, t0, te, a.k_hi));
  auto next = [&](const Pos& p) {
    Pos n = p;
    if (p.t >= te) return n;
    n.kk = p.kk + C::KC;
    if (n.kk >= int(pad_k(tri_ks(p.tri)))) {
      n.t = p.t + 1;
      n.kk = 0;
      if (n.t < te) n.tri = scalar_triple(a.tri, n.t);
    }
    return n;
  };
  Pos cur = {t0, 0, {0, 0}};
  if (t0 < te) cur.tri = uni(a.tri[t0]);
  if (cur.t < te) {
    load(cur.tri, 0, true, R0);
    store(R0, 0);
  }
  Pos p1 = next(cur);
  load(p1.tri, p1.kk, p1.t < te, R1);
  __syncthreads();

  // one chunk: read the fragments of stage `buf`, issue chunk c + 2 into Rn while they arrive,
  // run the MFMAs, then move chunk c + 1 from Ro into the other stage
  auto chunk = [&](Regs& Rn, Regs& Ro, int buf) {
    const bool triple_ends = cur.kk + C::KC >= int(pad_k(tri_ks(cur.tri)));
    const Pos p2 = next(p1);
    bf8 af[3][NRA], bfr[3][NCA];
    if constexpr (NR > 0 && NC > 0) {
      // rows 16 (rb0 + x) + i16 share (row >> 1) & 3 with i16, so one swizzled offset serves all
      const int fo = C::gpos(i16, g);
      const uint16_t* as = As + buf * C::ASZ + 16 * rb0 * C::RS + fo;
      const uint16_t* bs = Bs + buf * C::BSZ + 16 * cb0 * C::RS + fo;
#pragma unroll
      for (int s = 0; s < 3; ++s) {
#pragma unroll
        for (int x = 0; x < NR; ++x)
          af[s][x] = *reinterpret_cast<const bf8*>(as + s * TM * C::RS + 16 * x * C::RS);
#pragma unroll
        for (int y = 0; y < NC; ++y)
          bfr[s][y] = *reinterpret_cast<const bf8*>(bs + s * TN * C::RS + 16 * y * C::RS);
      }
    }
    load(p2.tri, p2.kk, p2.t < te, Rn);
    if constexpr (NR > 0 && NC > 0) {
      // the six slice products, smallest first; consecutive MFMAs hit different accumulators
      constexpr int PA[6] = {2, 1, 0, 1, 0, 0};
      constexpr int PB[6] = {0, 1, 2, 0, 1, 0};
#pragma unroll
      for (int m = 0; m < 6; ++m)
#pragma unroll
        for (int x = 0; x < NR; ++x)
#pragma unroll
          for (int y = 0; y < NC; ++y)
            acc32[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[PA[m]][x], bfr[PB[m]][y], acc32[x][y], 0, 0, 0);
      if (triple_ends) {
#pragma unroll
        for (int x = 0; x < NR; ++x)
#pragma unroll
          for (int y = 0; y < NC; ++y) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[x][y][r] += double(acc32[x][y][r]);
            acc32[x][y] = (f4){0.f, 0.f, 0.f, 0.f};
          }
      }
    }
    if (p1.t < te) store(Ro, buf ^ 1);
    __syncthreads();
    cur = p1;
    p1 = p2;
  };
  while (cur.t < te) {
    chunk(R0, R1, 0);
    if (cur.t >= te) break;
    chunk(R1, R0, 1);
  }

  // epilogue (v_mfma_f32_16x16x32_bf16: register r of lane 16g + i holds row 4g + r, column i)
  const double alpha = pa.alpha;
#pragma unroll
  for (int x = 0; x < NR; ++x)
#pragma unroll
    for (int y = 0; y < NC; ++y) {
      const int col = 16 * (cb0 + y) + i16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * (rb0 + x) + 4 * g + r;
        if (row < h && col < w) {
          const int64_t e = c_base + int64_t(row) * ldc + col;
          if (a.win_last) store_c(pa, e, alpha * acc[x][y][r], a.accumulate);
          else pa.P[e] = acc[x][y][r];
        }
      }
    }
}

// Selects the instantiation for the wave's rectangle shape among those the table holds.
template <int TM, int TN, int NW, bool RESUME, int NA, int NB>
__device__ __forceinline__ void dispatch_b3(int na, int nb, int rb0, int cb0, const TileArgs& a,
                                            const Item& it, const ProductArgs& pa, uint16_t* As,
                                            uint16_t* Bs) {
  constexpr int PA = TM / 16, PB = TN / 16;
  if constexpr (NA > PA) {
    return;
  } else if constexpr (NB > PB) {
    dispatch_b3<TM, TN, NW, RESUME, NA + 1, 0>(na, nb, rb0, cb0, a, it, pa, As, Bs);
  } else {
    if constexpr (WaveRects<PA, PB, NW>::used[NA][NB]) {
      if (na == NA && nb == NB) {
        run_b3<TM, TN, NW, RESUME, NA, NB>(a, it, pa, rb0, cb0, As, Bs);
        return;
      }
    }
    dispatch_b3<TM, TN, NW, RESUME, NA, NB + 1>(na, nb, rb0, cb0, a, it, pa, As, Bs);
  }
}

template <int TM, int TN, int KC, int NW, int OCC, bool RESUME>
__global__ __launch_bounds__(64 * NW, OCC) void tiles_bf16x3(TileArgs a) {
  using C = B3Cfg<TM, TN, NW>;
  static_assert(KC == kSliceK, "bf16 variant");
  __shared__ __attribute__((aligned(16))) uint16_t As[2 * C::ASZ];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2 * C::BSZ];
  const int x = blockIdx.x % kXcds, qx = blockIdx.x / kXcds;
  const int idx = a.map.begin[x] + qx;
  if (idx >= a.map.begin[x + 1] || idx == a.skip_task) return;
  if (a.stamps && threadIdx.x == 0) a.stamps[2 * idx] = wall_clock64();
  const Item it = uni(a.items[idx]);
  const ProductArgs pa = uni(a.prods ? a.prods[it.product] : a.single);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // this wave's rectangle of the sub-tile's output blocks (1 <= h <= TM, 1 <= w <= TN)
  const uint32_t rect = WaveRects<TM / 16, TN / 16, NW>::get((it.h + 15) >> 4, (it.w + 15) >> 4, wave);
  const int rb0 = int(rect & 0xFF), cb0 = int((rect >> 8) & 0xFF);
  const int na = int((rect >> 16) & 0xFF), nb = int(rect >> 24);
  dispatch_b3<TM, TN, NW, RESUME, 0, 0>(na, nb, rb0, cb0, a, it, pa, As, Bs);
  if (a.stamps) {
    __syncthreads();
    if (threadIdx.x == 0) a.stamps[2 * idx + 1] = wall_clock64();
  }
  if (threadIdx.x == 0) count_task(a.done, idx);
}

}  // namespace

hipError_t launch_tiles_bf16x3(int variant, int64_t grid, const TileArgs& args, hipStream_t stream) {
  if (grid <= 0) return hipSuccess;
  const uint32_t grid32 = static_cast<uint32_t>(grid);
#define BSM_B3_LAUNCH(ID, TM, TN, KC, NW, OCC)                                                    \
  case ID:                                                                                        \
    if (args.win_first)                                                                           \
      hipLaunchKernelGGL((tiles_bf16x3<TM, TN, KC, NW, OCC, false>), dim3(grid32), dim3(64 * NW), \
                         0, stream, args);                                                        \
    else                                                                                          \
      hipLaunchKernelGGL((tiles_bf16x3<TM, TN, KC, NW, OCC, true>), dim3(grid32), dim3(64 * NW),  \
                         0, stream, args);                                                        \
    break;
  switch (variant) {
    BSM_BF16_VARIANTS(BSM_B3_LAUNCH)
    default:
      return hipErrorInvalidValue;
  }
#undef BSM_B3_LAUNCH
  return hipGetLastError();
}

}  // namespace bsm
