// Launch wrappers of the device kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "types.hpp"

namespace bsm {

enum Form : int { FORM_F64 = 0, FORM_F32 = 1, FORM_BF16X3 = 2 };

constexpr int kNoKLimit = 1 << 30;

// Task range of each XCD: tasks begin[x] .. begin[x+1]-1 run on XCD x.
struct XcdMap {
  int32_t begin[kXcds + 1];
};

// Arguments of one tile-kernel launch.
struct TileArgs {
  const Item* items;
  const Triple* tri;
  XcdMap map;
  const ProductArgs* prods;  // per-product operands (batches); NULL = `single` for every task
  ProductArgs single;
  int accumulate;            // C = alpha*AB + C instead of C = alpha*AB (last window only)
  int k_lo, k_hi;            // only triples with k in [k_lo, k_hi) (k-window)
  int win_first, win_last;   // first window starts from 0, later ones from the partial sums
  uint64_t* stamps;          // 2 per task: start/end of the 100 MHz constant clock, or NULL
  uint32_t* done;            // per task: executions so far (checked by the host), or NULL
  int skip_task;             // task index the kernel leaves out (fault injection for tests), or -1
};

hipError_t launch_tiles_f64(int variant, int64_t grid, const TileArgs& args, hipStream_t stream);
hipError_t launch_tiles_f32(int variant, int64_t grid, const TileArgs& args, hipStream_t stream);

// The FP64/FP32 tile kernels are compiled one instantiation per translation unit
// (kernels_tile.hip, built once per form F = FORM_F64 / FORM_F32, variant ID and window kind R =
// 0 first / 1 later); each defines launch_tile_unit_<F>_<ID>_<R>.
#define BSM_DECLARE_TILE_UNITS(ID, TM, TN, KC, NW, OCC)                                 \
  hipError_t launch_tile_unit_0_##ID##_0(int64_t, const TileArgs&, hipStream_t);       \
  hipError_t launch_tile_unit_0_##ID##_1(int64_t, const TileArgs&, hipStream_t);       \
  hipError_t launch_tile_unit_1_##ID##_0(int64_t, const TileArgs&, hipStream_t);       \
  hipError_t launch_tile_unit_1_##ID##_1(int64_t, const TileArgs&, hipStream_t);
BSM_TILE_VARIANTS(BSM_DECLARE_TILE_UNITS)
#undef BSM_DECLARE_TILE_UNITS
// The split-bf16 tile kernel likewise (kernels_bf16x3.hip, once per variant ID and window kind R).
#define BSM_DECLARE_B3_UNITS(ID, TM, TN, KC, NW, OCC)                                  \
  hipError_t launch_b3_unit_##ID##_0(int64_t, const TileArgs&, hipStream_t);          \
  hipError_t launch_b3_unit_##ID##_1(int64_t, const TileArgs&, hipStream_t);
BSM_BF16_VARIANTS(BSM_DECLARE_B3_UNITS)
#undef BSM_DECLARE_B3_UNITS

// Device tables from which device-built k-lists are made (see klist.hip).
struct DevKlists {
  const uint64_t* a_bits;   // A's shape, M x wk words
  const uint64_t* bt_bits;  // B's shape transposed, N x wk words
  int64_t wk;
  const int64_t* a_tab;     // M x K packed offsets of A_ik (form's layout)
  const int64_t* bt_tab;    // N x K packed offsets of B_kj, at [j K + k]
  int64_t K;
  const int64_t* inner;     // inner block sizes
};

// Writes the k-list triples of njobs C blocks (KJob) into tri.
hipError_t launch_fill_klists(const KJob* jobs, int64_t njobs, const DevKlists& d, Triple* tri,
                              hipStream_t stream);

// dst[i] = src[i] rounded to FP32 for i < n.
hipError_t launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t stream);

// Three bf16 slices of every block of one operand (see SplitBlock), planes `plane` elements apart.
// stored blocks of a transposed operand -> the product's packed layout (FP64, or rounded to FP32)
hipError_t launch_transpose_f64(const XposeBlock* blocks, int64_t nblocks, const double* src,
                                double* dst, hipStream_t stream);
hipError_t launch_transpose_f32(const XposeBlock* blocks, int64_t nblocks, const double* src,
                                float* dst, hipStream_t stream);
// tensor blocks permuted element by element (matricization, and back for C); with accumulate the
// destination receives src + dst; dst is FP64 or (c_f32) FP32
hipError_t launch_permute_blocks(const PermBlock* blocks, int64_t nblocks, const double* src,
                                 void* dst, int c_f32, int accumulate, hipStream_t stream);
// reduction variant: dst[0 .. n) = 0, and C[e] = alpha sum_{s < S} P[s n + e] (+ C[e]) with the
// pieces added in order s = 0 .. S-1 (FP64; C FP64 or, with c_f32, rounded once to FP32)
hipError_t launch_fill_zero(double* dst, int64_t n, hipStream_t stream);
hipError_t launch_reduce_splits(const double* P, int S, int64_t n, void* C, int c_f32,
                                double alpha, int accumulate, hipStream_t stream);
// runs of elements src[src_off .. src_off + n) -> dst[dst_off ..), one workgroup per run
hipError_t launch_copy_blocks(const CopyBlock* blocks, int64_t nblocks, const double* src,
                              double* dst, hipStream_t stream);
// complex elements: the real embedding of the operands, and C = alpha [Re; Im] (+ C) as complex
hipError_t launch_embed_complex(const ZBlock* blocks, int64_t nblocks, const double* src,
                                double* dst, hipStream_t stream);
hipError_t launch_complex_epilogue(const ZCBlock* blocks, int64_t nblocks, const double* P,
                                   void* C, int c_f32, double ar, double ai, int accumulate,
                                   hipStream_t stream);
hipError_t launch_split_bf16x3(const SplitBlock* blocks, int64_t nblocks, const double* src,
                               uint16_t* dst, int64_t plane, hipStream_t stream);

hipError_t launch_tiles_bf16x3(int variant, int64_t grid, const TileArgs& args, hipStream_t stream);

// Task cost model network: kMlpIn features -> kMlpHidden -> kMlpHidden -> 1, ReLU.
constexpr int kMlpIn = 5, kMlpHidden = 32;
constexpr int kMlpParams = kMlpHidden * kMlpIn + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden +
                           kMlpHidden + 1;

// Affine maps around the network: x' = (x - fmean) / fstd on the way in, y' = y * tstd + tmean
// on the way out (identity: means 0, stds 1).
struct MlpNorm {
  float fmean[kMlpIn], fstd[kMlpIn];
  float tmean, tstd;
};

hipError_t launch_mlp_forward(const float* params, const float* X, int64_t n, float* Y,
                              const MlpNorm& norm, hipStream_t s);
// rows of per-chunk partial sums the gradient needs for n samples
int64_t mlp_partial_rows(int64_t n);
// grad (kMlpParams) and mean squared error loss over X (n x kMlpIn) against T (n); part must hold
// mlp_partial_rows(n) x kMlpParams floats, part_loss mlp_partial_rows(n) floats; loss may be NULL.
hipError_t launch_mlp_loss_grad(const float* params, const float* X, const float* T, int64_t n,
                                float* part, float* part_loss, float* grad, float* loss,
                                hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, int64_t step,
                       float lr, float b1, float b2, float eps, hipStream_t s);
// X[i][f] = (X[i][f] - mean[f]) / std[f], T[i] = (T[i] - tmean) / tstd, in place
hipError_t launch_mlp_normalize(float* X, float* T, int64_t n, const MlpNorm& norm, hipStream_t s);

}  // namespace bsm
