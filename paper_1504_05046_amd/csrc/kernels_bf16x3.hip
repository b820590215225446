// Split-bf16 tile contraction on gfx950 (v_mfma_f32_16x16x32_bf16).
//
// Each FP64 operand element is held as three bf16 slices a = a0 + a1 + a2 (written by the split
// pass).  A block product is formed from the six slice products of order <= 2,
//   a2 b0 + a1 b1 + a0 b2 + a1 b0 + a0 b1 + a0 b0,
// accumulated in FP32 inside one block product A_ik B_kj and added into FP64 registers when the
// triple ends; the epilogue writes alpha*sum (+C) once per element.
//
// One workgroup of NW waves runs one task (a C sub-tile of up to TM x TN and its k-list).  The
// k-list is streamed in 32-deep chunks, one MFMA step each (one k-panel of the slice planes, whose
// rows are contiguous).  The pipeline per chunk c:
//   * the chunk's three A and three B slice panels reach LDS by direct global->LDS loads
//     (buffer_load ... lds, 16 bytes per lane) issued two chunks ahead into a ring of three LDS
//     stages, so no staging registers and no LDS store instructions are needed;
//   * each wave reads its fragments of chunk c + 1 from LDS while its MFMAs of chunk c run from
//     the fragment registers read one chunk earlier (two fragment register sets), so LDS latency
//     is hidden behind the MFMAs;
//   * one barrier per chunk, after each wave has waited for its own loads of chunk c + 1 and for
//     its own fragment reads of chunk c: after it chunk c + 1 is complete in LDS for everyone and
//     chunk c's stage may be refilled (with chunk c + 3).
// The waits on the direct loads are explicit (s_waitcnt on the vector-memory counter); the
// barrier is a bare s_barrier between compiler-level memory barriers, because the workgroup fence
// of __syncthreads would wait for every load in flight, including the ones two chunks ahead.
//
// Each wave owns one rectangle of the sub-tile's 16x16 output blocks, from the same balanced
// table as the FP64/FP32 kernel.  With four waves a wave owns up to 4 x 4 blocks, so one 16-byte
// fragment read from LDS feeds up to 4 (slice-dependent: up to 12) MFMAs.
//
// LDS layout of a stage: per slice, one 64-byte row (32 bf16 of the k-panel) per A row or B
// column, no padding; the 16-byte granule o of row r sits at granule o ^ ((r >> 1) & 3).  Measured
// on gfx950 with the LDS bank-conflict counter, this makes the fragment reads (16 rows x 4
// granules per ds_read_b128) conflict-free.  A direct load writes 64 consecutive granules; each
// lane fetches the global granule that belongs at its position.
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

// s_waitcnt immediates (gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt in 6:4, lgkmcnt in
// 11:8; a field at its maximum is not waited on).
constexpr int vm_wait(int n) { return (n & 0xF) | (((n >> 4) & 3) << 14) | (0x7 << 4) | (0xF << 8); }
constexpr int kLgkmWait0 = 0xF | (0x3 << 14) | (0x7 << 4);

// A barrier that orders nothing but itself: the waits it needs are issued explicitly before it.
__device__ inline void bare_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

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
  static constexpr int KC = kSliceK;            // one MFMA step per chunk
  static constexpr int NT = 64 * NW;
  static constexpr int RS = KC;                 // LDS row: 32 bf16 = 64 bytes
  static constexpr int SLA = TM * RS, SLB = TN * RS;  // bf16 of one slice of a stage
  static constexpr int STAGE = 3 * (SLA + SLB); // bf16 of one stage (A then B)
  static constexpr int NSTAGE = 3;
  static constexpr int AG = 3 * TM * 4, BG = 3 * TN * 4;  // 16-byte granules of a stage
  static constexpr int ADMA = AG / NT, BDMA = BG / NT;    // direct loads per lane per stage
  static constexpr int DMA = ADMA + BDMA;
  static_assert(AG % NT == 0 && BG % NT == 0 && (TM * 4) % 64 == 0 && (TN * 4) % 64 == 0,
                "bf16 tile shape");
  static_assert(2 * DMA <= 63, "vector-memory counter range");
  // bf16 offset of granule o (8 bf16) of LDS row r
  __device__ static inline int gpos(int r, int o) { return r * RS + ((o ^ ((r >> 1) & 3)) << 3); }
};

using lds_ptr = __attribute__((address_space(3))) void*;

template <int TM, int TN, int NW, bool RESUME, int NR, int NC>
__device__ __forceinline__ void run_b3(const TileArgs& a, const Item& it, const ProductArgs& pa,
                                       int rb0, int cb0, uint16_t* L) {
  using C = B3Cfg<TM, TN, NW>;
  constexpr int NRA = NR > 0 ? NR : 1, NCA = NC > 0 ? NC : 1;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
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

  // Direct loads of one chunk into stage `st`.  Load q of this lane covers stage granule
  // G = (q NW + wave) 64 + lane of its operand: slice G / (rows 4), row (G mod rows 4) / 4, LDS
  // position G mod 4, which holds the row's granule (G mod 4) ^ ((row >> 1) & 3).  Rows past h
  // (columns past w) fall outside the descriptor and land as zeros; a chunk past the end of the
  // k-list goes through empty descriptors (zeros, no memory access).
  auto dma = [&](const Triple& t, int kk, bool valid, int st) {
    uint16_t* sbase = L + st * C::STAGE;
    const uint16_t* ab = Ag + tri_a_off(t) + int64_t(kk) * it.ldm + int64_t(it.r0) * kSliceK;
    const uint16_t* bb = Bg + tri_b_off(t) + int64_t(kk) * it.ldc + int64_t(it.c0) * kSliceK;
    const int na = uni(valid ? h * kSliceK * 2 : 0), nb = uni(valid ? w * kSliceK * 2 : 0);
#pragma unroll
    for (int q = 0; q < C::ADMA; ++q) {
      const int g0 = (q * NW + wave) * 64;              // first granule of this load (uniform)
      const int s = g0 / (TM * 4), r0g = g0 - s * (TM * 4);
      const int gr = r0g + lane, row = gr >> 2, o = (gr & 3) ^ ((row >> 1) & 3);
      const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
          uni_ptr(const_cast<uint16_t*>(ab + s * pa.a_plane)), (short)0, na, kRsrcWord3b);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr)(sbase + s * C::SLA + r0g * 8), 16,
                                               uint32_t((row * kSliceK + 8 * o) * 2), 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < C::BDMA; ++q) {
      const int g0 = (q * NW + wave) * 64;
      const int s = g0 / (TN * 4), r0g = g0 - s * (TN * 4);
      const int gr = r0g + lane, row = gr >> 2, o = (gr & 3) ^ ((row >> 1) & 3);
      const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
          uni_ptr(const_cast<uint16_t*>(bb + s * pa.b_plane)), (short)0, nb, kRsrcWord3b);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr)(sbase + 3 * C::SLA + s * C::SLB + r0g * 8),
                                               16, uint32_t((row * kSliceK + 8 * o) * 2), 0, 0, 0);
    }
  };

  // This wave's fragments of the chunk in stage `st`: for each slice, one A fragment per block row
  // and one B fragment per block column.  Rows 16 (rb0 + x) + i16 share (row >> 1) & 3 with i16,
  // so one swizzled offset serves all of them.
  struct Frags {
    bf8 a[3][NRA], b[3][NCA];
  };
  auto read = [&](Frags& F, int st) {
    if constexpr (NR > 0 && NC > 0) {
      const int fo = C::gpos(i16, g);
      const uint16_t* as = L + st * C::STAGE + 16 * rb0 * C::RS + fo;
      const uint16_t* bs = L + st * C::STAGE + 3 * C::SLA + 16 * cb0 * C::RS + fo;
#pragma unroll
      for (int s = 0; s < 3; ++s) {
#pragma unroll
        for (int x = 0; x < NR; ++x)
          F.a[s][x] = *reinterpret_cast<const bf8*>(as + s * C::SLA + 16 * x * C::RS);
#pragma unroll
        for (int y = 0; y < NC; ++y)
          F.b[s][y] = *reinterpret_cast<const bf8*>(bs + s * C::SLB + 16 * y * C::RS);
      }
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

  // prologue: chunks 0, 1, 2 into stages 0, 1, 2; fragments of chunk 0
  Pos cur = {t0, 0, {0, 0}};
  if (t0 < te) cur.tri = scalar_triple(a.tri, t0);
  Pos p1 = next(cur);
  Pos p2 = next(p1);
  dma(cur.tri, cur.kk, cur.t < te, 0);
  dma(p1.tri, p1.kk, p1.t < te, 1);
  dma(p2.tri, p2.kk, p2.t < te, 2);
  __builtin_amdgcn_s_waitcnt(vm_wait(2 * C::DMA));
  bare_barrier();
  Frags F0, F1;
  read(F0, 0);

  // one chunk: MFMAs from Fc while Fn receives chunk c + 1's fragments; `st` is chunk c's stage
  int st = 0;
  auto chunk = [&](Frags& Fc, Frags& Fn) {
    const Pos p3 = next(p2);
    const bool triple_ends = cur.kk + C::KC >= int(pad_k(tri_ks(cur.tri)));
    __builtin_amdgcn_s_waitcnt(kLgkmWait0);        // own fragment reads of chunk c are done
    __builtin_amdgcn_s_waitcnt(vm_wait(C::DMA));   // own loads of chunk c + 1 have landed
    bare_barrier();
    dma(p3.tri, p3.kk, p3.t < te, st);             // chunk c + 3 into chunk c's stage
    const int st1 = st == 2 ? 0 : st + 1;
    read(Fn, st1);
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
            acc32[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Fc.a[PA[m]][x], Fc.b[PB[m]][y],
                                                                  acc32[x][y], 0, 0, 0);
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
    st = st1;
    cur = p1;
    p1 = p2;
    p2 = p3;
  };
  while (cur.t < te) {
    chunk(F0, F1);
    if (cur.t >= te) break;
    chunk(F1, F0);
  }
  // every direct load (the prefetches past the end included) has landed before the workgroup
  // may exit and its LDS be reused
  __builtin_amdgcn_s_waitcnt(vm_wait(0));

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
                                            const Item& it, const ProductArgs& pa, uint16_t* L) {
  constexpr int PA = TM / 16, PB = TN / 16;
  if constexpr (NA > PA) {
    return;
  } else if constexpr (NB > PB) {
    dispatch_b3<TM, TN, NW, RESUME, NA + 1, 0>(na, nb, rb0, cb0, a, it, pa, L);
  } else {
    if constexpr (WaveRects<PA, PB, NW>::used[NA][NB]) {
      if (na == NA && nb == NB) {
        run_b3<TM, TN, NW, RESUME, NA, NB>(a, it, pa, rb0, cb0, L);
        return;
      }
    }
    dispatch_b3<TM, TN, NW, RESUME, NA, NB + 1>(na, nb, rb0, cb0, a, it, pa, L);
  }
}

template <int TM, int TN, int KC, int NW, int OCC, bool RESUME>
__global__ __launch_bounds__(64 * NW, OCC) void tiles_bf16x3(TileArgs a) {
  using C = B3Cfg<TM, TN, NW>;
  static_assert(KC == kSliceK, "bf16 variant");
  __shared__ __attribute__((aligned(16))) uint16_t L[C::NSTAGE * C::STAGE];
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
  dispatch_b3<TM, TN, NW, RESUME, 0, 0>(na, nb, rb0, cb0, a, it, pa, L);
  if (a.stamps) {
    __syncthreads();
    if (threadIdx.x == 0) a.stamps[2 * idx + 1] = wall_clock64();
  }
  if (threadIdx.x == 0) count_task(a.done, idx);
}

}  // namespace

// One instantiation per translation unit (built once per variant BSM_B3_UNIT_ID and window kind
// BSM_B3_UNIT_RESUME, 0 = first k-window, 1 = a later one); launch_tiles_bf16x3 in
// tile_dispatch.hip picks among them.  Without the two macros this unit defines no launcher.
#if defined(BSM_B3_UNIT_ID) && defined(BSM_B3_UNIT_RESUME)
template <int ID>
struct B3Row;
#define BSM_B3_ROW_TRAITS(ID_, TM_, TN_, KC_, NW_, OCC_)                  \
  template <>                                                          \
  struct B3Row<ID_> {                                                  \
    static constexpr int TM = TM_, TN = TN_, KC = KC_, NW = NW_, OCC = OCC_; \
  };
BSM_BF16_VARIANTS(BSM_B3_ROW_TRAITS)
#undef BSM_B3_ROW_TRAITS
#define BSM_B3_NAME2(I, R) launch_b3_unit_##I##_##R
#define BSM_B3_NAME(I, R) BSM_B3_NAME2(I, R)
hipError_t BSM_B3_NAME(BSM_B3_UNIT_ID, BSM_B3_UNIT_RESUME)(int64_t grid, const TileArgs& args,
                                                           hipStream_t stream) {
  using R = B3Row<BSM_B3_UNIT_ID>;
  hipLaunchKernelGGL((tiles_bf16x3<R::TM, R::TN, R::KC, R::NW, R::OCC, BSM_B3_UNIT_RESUME != 0>),
                     dim3(static_cast<uint32_t>(grid)), dim3(64 * R::NW), 0, stream, args);
  return hipGetLastError();
}
#endif

}  // namespace bsm
