// Task and operand descriptors shared by the host planner and the device kernels.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define BSM_HD __host__ __device__
#else
#define BSM_HD
#endif

namespace bsm {

// Limits that the packed descriptors impose.
constexpr int64_t kMaxBlock = 65535;          // block sizes fit 16 bits
constexpr int64_t kMaxElems = int64_t(1) << 48;  // tile offsets fit 48 bits
constexpr int kXcds = 8;                       // MI355X: 8 accelerator dies, each with its own L2

// Tile variants: X(id, TM, TN, KC, NW, OCC) = largest C sub-tile TM x TN of one workgroup,
// k-chunk KC staged through LDS per step, NW waves per workgroup, OCC waves per SIMD the register
// allocator must leave room for (512 / OCC registers per lane).  Sub-tiles are cut in multiples
// of 16 rows/columns.
#define BSM_TILE_VARIANTS(X)    \
  X(0, 128, 128, 16, 8, 4)      \
  X(1, 128, 128, 16, 4, 2)      \
  X(2, 64, 64, 16, 4, 3)        \
  X(3, 32, 32, 16, 4, 4)

// Split-bf16 tile variants (same fields; the k-chunk is one 32-deep bf16 MFMA step): 128 x 128
// with 8 waves (two per SIMD) or 4 waves (one per SIMD, 4 x 4 blocks per wave), both with 144 KB
// of LDS, and 64 x 64 with two workgroups per CU.
#define BSM_BF16_VARIANTS(X) \
  X(0, 128, 128, 32, 8, 2)   \
  X(1, 128, 128, 32, 4, 1)   \
  X(2, 64, 64, 32, 4, 2)

// Slice planes of the split-bf16 form: each block with its inner size padded to a multiple of 32
// (zeros), A blocks as rows x s32 and B blocks transposed (cols x s32), so that both MFMA operands
// read 8 consecutive k per lane.  Within a block the 32-wide k-panels are stored one after the
// other, each panel row-major (rows x 32): element (r, k) of a block of R rows sits at
// (k / 32) * 32 R + 32 r + k % 32, so that the rows of one k-chunk are contiguous in memory.
constexpr int kSliceK = 32;
BSM_HD inline int64_t pad_k(int64_t ks) { return (ks + kSliceK - 1) / kSliceK * kSliceK; }

// One piece of an operand block as the split pass sees it (the planner cuts each block into its
// 32-wide k-panels): src_off in the packed FP64 tiles, dst_off in a slice plane, `rows` output
// rows (A rows, or B columns when transposed), inner size ks of the piece.
struct SplitBlock {
  int64_t src_off;
  int64_t dst_off;
  int32_t rows;
  int32_t ks;
  int32_t ld_src;     // leading dimension of the source block (ks for A, the B block's width)
  int32_t transpose;  // 1: the source is ks x rows (B) and is written transposed
};

// One piece of a transposition pass (a transposed operand into the product's layout, V factors
// into V^T, a tensor block whose modes fall into two swapped groups): rows x cols source elements,
// element (r, c) at src_off + r ld_src + c, written to dst_off + c ld_dst + r.  Large blocks are
// cut into bands of rows so that one workgroup handles one band.
struct XposeBlock {
  int64_t src_off;
  int64_t dst_off;
  int32_t rows;
  int32_t cols;
  int32_t ld_src;
  int32_t ld_dst;
};

// One contiguous run of n elements copied from src_off to dst_off (gathering the dense blocks and
// U factors of a block-rank-sparse operand into an ordinary packed operand).
struct CopyBlock {
  int64_t src_off;
  int64_t dst_off;
  int64_t n;
};

// One block of a tensor operand as the permutation pass sees it: the source block is row-major
// over its `order` modes with extents ext (last mode fastest); element (x_0 .. x_{d-1}) goes to
// dst_off + sum_m x_m dst_stride[m] (the matricized block's, or the tensor block's, row-major
// position).
constexpr int kMaxModes = 8;
// Source elements [e0, e1) of the block (a large block is cut into several pieces).
struct PermBlock {
  int64_t src_off;
  int64_t dst_off;
  int32_t order;
  int32_t pad_;
  int32_t ext[kMaxModes];
  int64_t dst_stride[kMaxModes];
  int64_t e0, e1;
};

// Complex elements run as a real product: one piece of a block of a complex operand as the
// embedding pass sees it.  The op(X) block is full_rows x cols complex elements; a piece is `rows`
// of its rows (the planner cuts blocks into bands of kZBand rows), src_off and dst_off already
// point at the piece's first row.  src_off counts complex elements of the caller's buffer, dst_off
// real elements of the embedded operand.  mode: bit 0 = stored transposed (the source block is
// cols x full_rows), bit 1 = conjugate, bit 2 = right operand (written as the 2 full_rows x cols
// real block [Re; Im]; otherwise the 2 full_rows x 2 cols block [[Re, -Im], [Im, Re]]); full_rows
// places the imaginary half and is the row pitch of a transposed source.
struct ZBlock {
  int64_t src_off;
  int64_t dst_off;
  int32_t rows;
  int32_t cols;
  int32_t mode;
  int32_t full_rows;
};
constexpr int kZTrans = 1, kZConj = 2, kZRight = 4;
constexpr int kZBand = 32;         // complex rows per embedding piece
constexpr int64_t kZCPiece = 1 << 14;  // complex elements per epilogue piece

// One piece of a complex C block for the epilogue: the block's offset (complex elements; the real
// product's [Re; Im] block starts at 2 off) and element count n, and the piece's elements
// [e0, e1) of it.
struct ZCBlock {
  int64_t off;
  int64_t n;
  int64_t e0, e1;
};

// One (i,k,j) block triple of a C block's k-list: where A_ik and B_kj start and the inner block
// size.  a = A offset | (s_k << 48);  b = B offset | (k << 48).
struct Triple {
  uint64_t a;
  uint64_t b;
};

BSM_HD inline int64_t tri_a_off(const Triple& t) { return int64_t(t.a & 0xFFFFFFFFFFFFull); }
BSM_HD inline int tri_ks(const Triple& t) { return int(t.a >> 48); }
BSM_HD inline int64_t tri_b_off(const Triple& t) { return int64_t(t.b & 0xFFFFFFFFFFFFull); }
BSM_HD inline int tri_k(const Triple& t) { return int(t.b >> 48); }

// One task: a sub-tile (rows r0..r0+h, cols c0..c0+w) of the C block at c_off (a block of
// `ldc` columns), and its k-list tri[tri_begin .. tri_begin + tri_count).
struct Item {
  int64_t c_off;
  uint32_t tri_begin;
  uint32_t tri_count;
  uint16_t r0, c0, h, w;
  uint16_t ldc;       // C block width = width of every B_kj of the k-list
  uint16_t ldm;       // C block height = height of every A_ik of the k-list
  uint32_t product;   // index into the batch's operand table (0 for a single product)
};
static_assert(sizeof(Item) == 32, "Item layout");

// Device-built k-list of one C block (i, j): the triples of its k-list, ascending k, are written
// at tri[tri_begin .. tri_begin + count) before the tile kernel of the batch runs.
struct KJob {
  int32_t i, j;
  uint32_t tri_begin, count;
};

// Operands of one product: A and B in the element type of the precision form (FP64 tiles, or
// their FP32 / bf16-slice copies), C in FP64 or FP32 (c_f32) and the k-window partial sums P in
// FP64.
struct ProductArgs {
  const void* A;
  const void* B;
  void* C;
  double* P;
  double alpha;
  int64_t a_plane, b_plane;  // split-bf16 form: elements between consecutive slice planes
  int32_t c_f32;             // 1: C holds FP32 elements
  int32_t pad_;
};

}  // namespace bsm
