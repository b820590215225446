// Tile contraction on gfx950 MFMA, FP64 and FP32 forms.
//
// One workgroup (NW waves) executes one task: a C sub-tile of h x w (h <= TM, w <= TN) and the
// k-list of its C block (the triples whose k lies in the current k-window).  For every triple, in
// ascending k, the workgroup streams KC-wide k-chunks of A_ik (rows r0..r0+h) and B_kj (cols
// c0..c0+w) from HBM into LDS (double-buffered, one barrier per chunk; the loads run two chunks
// ahead through two sets of staging registers).  Each wave owns a rectangle of na x nb of the
// sub-tile's 16x16 output blocks (a generated table, balanced across the waves), so that one
// 4-deep MFMA step reads na + nb fragments from LDS for na * nb MFMAs.  FP64 form:
// v_mfma_f64_16x16x4 into FP64 registers across the whole k-list.  FP32 form: v_mfma_f32_16x16x4 into FP32 registers within
// one block product A_ik B_kj, folded into FP64 registers when the triple ends.  The epilogue
// writes alpha*acc (+C) once per element: the paper's multiply task and reduction task fused,
// with no temporaries (Sec. 3.2, Fig. 3).
#include <hip/hip_runtime.h>

#pragma once
#include "kernels.hpp"
#include "uniform.hpp"
#include "wave_rects.inc"

namespace bsm {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

// Fourth word of a raw (stride 0) buffer descriptor on gfx9-family targets: 32-bit data format,
// no swizzle; loads past num_records return 0.
constexpr int kRsrcWord3 = 0x00020000;
constexpr uint32_t kOutOfRange = 0x7FFFFFF0u;

template <int FORM>
struct FormT;

template <>
struct FormT<FORM_F64> {
  using T = double;
  static constexpr bool kFold = false;
  __device__ static inline T load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  }
  // v_mfma_f64_16x16x4: register r of lane 16g + i holds row g + 4r, column i (gfx950)
  __device__ static inline int out_row(int g, int r) { return g + 4 * r; }
};

template <>
struct FormT<FORM_F32> {
  using T = float;
  static constexpr bool kFold = true;
  __device__ static inline T load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  }
  // v_mfma_f32_16x16x4: register r of lane 16g + i holds row 4g + r, column i
  __device__ static inline int out_row(int g, int r) { return 4 * g + r; }
};

template <int TM, int TN, int KC_, int NW_, int FORM>
struct TileCfg {
  using T = typename FormT<FORM>::T;
  static constexpr int ES = int(sizeof(T));
  static constexpr int KC = KC_;            // k-chunk staged per step
  static constexpr int NW = NW_;            // waves per workgroup
  static constexpr int NT = 64 * NW;        // threads per workgroup
  // A chunk (TM rows x KC) in LDS, step-major: k = 4s + g (s = MFMA step, g = lane group) is
  // stored at s * APL + 4 row + (g ^ 2 * bit3(row)), planes APL = 4 TM + 8 apart.  The XOR on g
  // separates rows r and r + 8, so a half-wave's fragment reads (16 rows, two g) hit distinct
  // banks; the 8-element plane padding does the same for the staging stores (two rows, all s);
  // and every step's reads sit at a compile-time offset from one per-lane address.
  static constexpr int APL = 4 * TM + 8;
  __device__ static inline int apos(int row, int k) {
    return (k >> 2) * APL + 4 * row + ((k & 3) ^ (((row >> 3) & 1) << 1));
  }
  // B chunk: KC rows x TN, padded so that a half-wave's fragment reads hit distinct banks
  static constexpr int BSTR = TN + 16;
  static constexpr int PA = TM / 16, PB = TN / 16;  // 16x16 output blocks per sub-tile side
  static constexpr int ARP = NT / KC;       // A rows staged per pass (KC threads per row)
  static constexpr int ALD = TM / ARP;      // A elements each thread stages per chunk
  static constexpr int BK = NT / TN;        // B k-rows staged per pass (TN threads per row)
  static constexpr int BLD = KC / BK;       // B elements each thread stages per chunk
  static constexpr int ASZ = (KC / 4) * APL;  // elements of one A stage
  static constexpr int BSZ = KC * BSTR;     // elements of one B stage
  static_assert(KC % 16 == 0 && NT % KC == 0 && TM % ARP == 0, "A staging shape");
  static_assert(TN <= NT && NT % TN == 0 && KC % BK == 0, "B staging shape");
};

// First triple of [tb, te) whose inner block index is >= k (the k-lists are sorted by k).
__device__ inline uint32_t lower_bound_k(const Triple* __restrict__ tri, uint32_t tb, uint32_t te,
                                         int k) {
  while (tb < te) {
    uint32_t mid = tb + ((te - tb) >> 1);
    if (tri_k(tri[mid]) < k) tb = mid + 1;
    else te = mid;
  }
  return tb;
}

// The part of a task one wave runs when it owns the NA x NB output blocks whose top-left block
// is (rb0, cb0); block j = x NB + y is (rb0 + x, cb0 + y).  Every wave of the workgroup walks the
// same k-chunks and meets the same barriers; NA and NB are compile-time constants so that the
// MFMA stream has no per-block branches.
template <int TM, int TN, int KC, int NW, int FORM, bool RESUME, int NA, int NB>
__device__ __forceinline__ void run_task(const TileArgs& a, const Item& it, const ProductArgs& pa,
                                         int rb0, int cb0, typename FormT<FORM>::T* As,
                                         typename FormT<FORM>::T* Bs) {
  using C = TileCfg<TM, TN, KC, NW, FORM>;
  using F = FormT<FORM>;
  using T = typename C::T;
  constexpr int NS = NA * NB;
  constexpr int NSA = NS > 0 ? NS : 1;
  const int tid = threadIdx.x, lane = tid & 63;
  const int g = lane >> 4, i16 = lane & 15;
  const int h = it.h, w = it.w, ldc = it.ldc;

  // LDS offsets of this wave's A fragments (per block row) and B fragments (per block column)
  int a_u[NA > 0 ? NA : 1], b_u[NB > 0 ? NB : 1];
#pragma unroll
  for (int x = 0; x < NA; ++x) a_u[x] = 64 * (rb0 + x);
#pragma unroll
  for (int y = 0; y < NB; ++y) b_u[y] = 16 * (cb0 + y);
  const int64_t c_base = it.c_off + int64_t(it.r0) * ldc + it.c0;

  // FP64 accumulators; with a k-window after the first they resume from the raw partial sums
  // (a separate instantiation, so that the common single-window case carries none of it)
  d4 acc[NSA];
  const __amdgpu_buffer_rsrc_t prs = __builtin_amdgcn_make_buffer_rsrc(
      uni_ptr(pa.P + c_base), (short)0, uni(RESUME ? ((h - 1) * ldc + w) * 8 : 0), kRsrcWord3);
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    acc[j] = (d4){0.0, 0.0, 0.0, 0.0};
    if constexpr (RESUME) {
      const int rbk = rb0 + j / (NB > 0 ? NB : 1), cbk = cb0 + j % (NB > 0 ? NB : 1);
      const int col = 16 * cbk + i16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = 16 * rbk + F::out_row(g, r);
        uint32_t off = (row < h && col < w) ? uint32_t((row * ldc + col) * 8) : kOutOfRange;
        acc[j][r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(prs, off, 0, 0));
      }
    }
  }
  f4 acc32[FORM == FORM_F32 ? NSA : 1];
  if constexpr (FORM == FORM_F32) {
#pragma unroll
    for (int j = 0; j < NS; ++j) acc32[j] = (f4){0.f, 0.f, 0.f, 0.f};
  }

  // staging assignment: A chunk row-major (KC consecutive threads read one row's k-chunk),
  // B chunk row-major (TN consecutive threads read one k-row's columns)
  const int ka = tid % KC, ra0 = tid / KC;
  const int cbl = tid % TN, kb0 = tid / TN;
  const T* Ag = static_cast<const T*>(pa.A);
  const T* Bg = static_cast<const T*>(pa.B);

  // Two sets of staging registers: while chunk c is computed from LDS, the loads of chunk c + 2
  // are in flight into one set and chunk c + 1 waits in the other for its turn in LDS.
  struct Regs {
    T a[C::ALD], b[C::BLD];
  };
  Regs R0, R1;

  // Staging loads go through buffer descriptors: a load whose offset lies past num_records
  // returns 0 instead of touching memory.  A's descriptor ends at row h of the sub-tile, so rows
  // beyond it read 0; the k-tail (k >= s_k would wrap into the next row) is sent out of range
  // explicitly.  B's descriptor starts at the chunk's first k-row (64-bit base, so offsets stay
  // below KC rows of the block whatever its size) and ends at the last element of the sub-tile's
  // columns in the chunk's last k-row below s_k, so k-rows beyond s_k read 0; columns beyond w
  // read finite neighbours that only feed output columns the epilogue discards.  A chunk past
  // the end of the k-list is loaded with empty descriptors (zeros, no memory access), so that
  // every chunk issues the same loads.
  constexpr int NPART = C::KC / 4;
  auto load = [&](const Triple& t, int kk, bool valid, Regs& R, int part) {
    const int ks = tri_ks(t);
    const __amdgpu_buffer_rsrc_t ar = __builtin_amdgcn_make_buffer_rsrc(
        uni_ptr(const_cast<T*>(Ag + tri_a_off(t) + int64_t(it.r0) * ks)), (short)0,
        uni(valid ? h * ks * C::ES : 0), kRsrcWord3);
    const int krows = min(C::KC, ks - kk);  // k-rows of B_kj in this chunk (>= 1 when valid)
    const __amdgpu_buffer_rsrc_t br = __builtin_amdgcn_make_buffer_rsrc(
        uni_ptr(const_cast<T*>(Bg + tri_b_off(t) + int64_t(kk) * ldc + it.c0)), (short)0,
        uni(valid ? ((krows - 1) * ldc + w) * C::ES : 0), kRsrcWord3);
    const bool kin = kk + ka < ks;
#pragma unroll
    for (int p = 0; p < C::ALD; ++p) {
      if (part < 0 || p % NPART == part) {
        const uint32_t off = kin ? uint32_t(((ra0 + C::ARP * p) * ks + kk + ka) * C::ES) : kOutOfRange;
        R.a[p] = F::load(ar, off);
      }
    }
#pragma unroll
    for (int p = 0; p < C::BLD; ++p) {
      if (part < 0 || p % NPART == part) {
        const uint32_t off = uint32_t(((kb0 + C::BK * p) * ldc + cbl) * C::ES);
        R.b[p] = F::load(br, off);
      }
    }
  };
  auto store = [&](const Regs& R, int buf) {
    T* as = As + buf * C::ASZ;
    T* bs = Bs + buf * C::BSZ;
#pragma unroll
    for (int p = 0; p < C::ALD; ++p) as[C::apos(ra0 + C::ARP * p, ka)] = R.a[p];
#pragma unroll
    for (int p = 0; p < C::BLD; ++p) bs[(kb0 + C::BK * p) * C::BSTR + cbl] = R.b[p];
  };

  // A chunk's place in the k-list: triple index t (valid while t < te), its triple, and the
  // offset kk of the chunk within the block's inner dimension.
  struct Pos {
    uint32_t t;
    int kk;
    Triple tri;
  };
  uint32_t te = it.tri_begin + it.tri_count;
  uint32_t t0 = it.tri_begin;
  if (a.k_lo > 0) t0 = uni(lower_bound_k(a.tri, t0, te, a.k_lo));
  if (a.k_hi < kNoKLimit) te = uni(lower_bound_k(a.tri, t0, te, a.k_hi));
  // the chunk after p: the rest of p's block, else the next triple's first chunk
  auto next = [&](const Pos& p) {
    Pos n = p;
    if (p.t >= te) return n;
    n.kk = p.kk + C::KC;
    if (n.kk >= tri_ks(p.tri)) {
      n.t = p.t + 1;
      n.kk = 0;
      if (n.t < te) n.tri = uni(a.tri[n.t]);
    }
    return n;
  };
  Pos cur = {t0, 0, {0, 0}};
  if (t0 < te) cur.tri = uni(a.tri[t0]);
  if (cur.t < te) {
    load(cur.tri, 0, true, R0, -1);
    store(R0, 0);
  }
  Pos p1 = next(cur);
  load(p1.tri, p1.kk, p1.t < te, R1, -1);
  __syncthreads();

  // one chunk: compute from LDS stage `buf`; issue chunk c + 2 into Rn; move chunk c + 1 from Ro
  // into the other stage
  auto chunk = [&](Regs& Rn, Regs& Ro, int buf) {
    const int ks = tri_ks(cur.tri);
    const int nsteps = (min(C::KC, ks - cur.kk) + 3) >> 2;  // 4-deep MFMA steps holding data
    const bool triple_ends = cur.kk + C::KC >= ks;
    const Pos p2 = next(p1);

    {
      const T* as = As + buf * C::ASZ;
      const T* bs = Bs + buf * C::BSZ + g * C::BSTR + i16;
      // one 4-deep MFMA step per iteration: NA A fragments and NB B fragments, then the NA x NB
      // products; steps past the block's end hold only zeros and are skipped (the condition is the
      // same for the whole wave)
#pragma unroll
      for (int s = 0; s < C::KC / 4; ++s) {
        // step s reads its fragments, part s of chunk c + 2's loads goes out while they arrive,
        // then the MFMAs
        T av[NA > 0 ? NA : 1], bv[NB > 0 ? NB : 1];
        if (NS > 0 && s < nsteps) {
#pragma unroll
          for (int x = 0; x < NA; ++x) av[x] = as[a_u[x] + C::apos(i16, 4 * s + g)];
#pragma unroll
          for (int y = 0; y < NB; ++y) bv[y] = bs[b_u[y] + 4 * s * C::BSTR];
        }
        load(p2.tri, p2.kk, p2.t < te, Rn, s);
        if (NS > 0 && s < nsteps) {
#pragma unroll
          for (int x = 0; x < NA; ++x) {
#pragma unroll
            for (int y = 0; y < NB; ++y) {
              if constexpr (FORM == FORM_F64)
                acc[x * NB + y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[y], acc[x * NB + y], 0, 0, 0);
              else
                acc32[x * NB + y] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[x], bv[y], acc32[x * NB + y], 0, 0, 0);
            }
          }
        }
      }
      if constexpr (F::kFold) {
        // the block product A_ik B_kj is complete: add it to the FP64 sum across k
        if (NS > 0 && triple_ends) {
#pragma unroll
          for (int j = 0; j < NS; ++j) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[j][r] += double(acc32[j][r]);
            acc32[j] = (f4){0.f, 0.f, 0.f, 0.f};
          }
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

  // epilogue: the raw sum goes to the partial buffer until the last k-window, which writes
  // alpha*sum (+C)
  const double alpha = pa.alpha;
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const int rbk = rb0 + j / (NB > 0 ? NB : 1), cbk = cb0 + j % (NB > 0 ? NB : 1);
    const int col = 16 * cbk + i16;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int row = 16 * rbk + F::out_row(g, r);
      if (row < h && col < w) {
        const int64_t e = c_base + int64_t(row) * ldc + col;
        if (a.win_last) store_c(pa, e, alpha * acc[j][r], a.accumulate);
        else pa.P[e] = acc[j][r];
      }
    }
  }
}

// Selects the instantiation for the wave's rectangle shape among those the table holds.
template <int TM, int TN, int KC, int NW, int FORM, bool RESUME, int NA, int NB>
__device__ __forceinline__ void dispatch_rect(int na, int nb, int rb0, int cb0, const TileArgs& a,
                                              const Item& it, const ProductArgs& pa,
                                              typename FormT<FORM>::T* As,
                                              typename FormT<FORM>::T* Bs) {
  constexpr int PA = TM / 16, PB = TN / 16;
  if constexpr (NA > PA) {
    return;
  } else if constexpr (NB > PB) {
    dispatch_rect<TM, TN, KC, NW, FORM, RESUME, NA + 1, 0>(na, nb, rb0, cb0, a, it, pa, As, Bs);
  } else {
    if constexpr (WaveRects<PA, PB, NW>::used[NA][NB]) {
      if (na == NA && nb == NB) {
        run_task<TM, TN, KC, NW, FORM, RESUME, NA, NB>(a, it, pa, rb0, cb0, As, Bs);
        return;
      }
    }
    dispatch_rect<TM, TN, KC, NW, FORM, RESUME, NA, NB + 1>(na, nb, rb0, cb0, a, it, pa, As, Bs);
  }
}

template <int TM, int TN, int KC, int NW, int OCC, int FORM, bool RESUME>
__global__ __launch_bounds__(64 * NW, OCC) void tiles(TileArgs a) {
  using C = TileCfg<TM, TN, KC, NW, FORM>;
  using T = typename C::T;
  __shared__ T As[2 * C::ASZ];
  __shared__ T Bs[2 * C::BSZ];

  // XCD-aware task lookup: the hardware deals workgroups round-robin over the 8 XCDs, so
  // workgroup 8q + x runs on XCD x and takes that XCD's q-th task.
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
  dispatch_rect<TM, TN, KC, NW, FORM, RESUME, 0, 0>(na, nb, rb0, cb0, a, it, pa, As, Bs);
  if (a.stamps) {
    __syncthreads();
    if (threadIdx.x == 0) a.stamps[2 * idx + 1] = wall_clock64();
  }
  if (threadIdx.x == 0) count_task(a.done, idx);
}

// One tile-kernel instantiation: variant row ID of BSM_TILE_VARIANTS, precision form FORM,
// first window (RESUME = false) or a later one.
template <int ID>
struct VariantRow;
#define BSM_VARIANT_ROW_TRAITS(ID_, TM_, TN_, KC_, NW_, OCC_)                          \
  template <>                                                                        \
  struct VariantRow<ID_> {                                                           \
    static constexpr int TM = TM_, TN = TN_, KC = KC_, NW = NW_, OCC = OCC_;         \
  };
BSM_TILE_VARIANTS(BSM_VARIANT_ROW_TRAITS)
#undef BSM_VARIANT_ROW_TRAITS

template <int ID, int FORM, bool RESUME>
hipError_t launch_tile_instance(int64_t grid, const TileArgs& args, hipStream_t stream) {
  using R = VariantRow<ID>;
  hipLaunchKernelGGL((tiles<R::TM, R::TN, R::KC, R::NW, R::OCC, FORM, RESUME>),
                     dim3(static_cast<uint32_t>(grid)), dim3(64 * R::NW), 0, stream, args);
  return hipGetLastError();
}

}  // namespace bsm
