// Host planner: validation, C-shape, packing offsets, task expansion and task order.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "types.hpp"

namespace bsm {

// Tile variants (see BSM_TILE_VARIANTS): the largest C sub-tile one workgroup computes.
struct Variant {
  int tm, tn, nw;
};
#define BSM_VARIANT_ROW(ID, TM, TN, KC, NW, OCC) {TM, TN, NW},
constexpr Variant kVariants[] = {BSM_TILE_VARIANTS(BSM_VARIANT_ROW)};
constexpr int kNumVariants = int(sizeof(kVariants) / sizeof(kVariants[0]));
constexpr int kDefaultVariant = 0;  // 128 x 128, 8 waves
constexpr Variant kBf16Variants[] = {BSM_BF16_VARIANTS(BSM_VARIANT_ROW)};
constexpr int kNumBf16Variants = int(sizeof(kBf16Variants) / sizeof(kBf16Variants[0]));
constexpr int kDefaultBf16Variant = 0;
#undef BSM_VARIANT_ROW

// Task order: LOCALITY keeps C-block order and cuts it into one contiguous run per XCD; LPT sorts
// by cost and bins greedily; INTERLEAVE deals whole C blocks, in C-block order, each to the
// least-loaded XCD, so that all XCDs work on the same region of C at the same time; PATCH deals
// whole rectangles of patch_r x patch_c C blocks, so that the tasks an XCD runs together share
// few A block rows and B block columns in its L2.
enum Order : int {
  ORDER_LOCALITY = 0,
  ORDER_LPT = 1,
  ORDER_INTERLEAVE = 2,
  ORDER_PATCH = 3,
  ORDER_AUTO = 4  // LPT for up to kLptTasks tasks, INTERLEAVE above
};
// Task count up to which the automatic order deals largest-first: with few tasks per XCD the
// tail of the schedule decides the makespan (measured 16-23 % faster than the interleaved order
// at 900-4600 tasks of very uneven size); with many tasks the interleaved order keeps each XCD's
// concurrent tasks on neighbouring C blocks (5 % faster at 32000 tasks).
constexpr size_t kLptTasks = 8192;

struct PlanConfig {
  int precision = 0;
  int sched = 0;
  int64_t k_window = 0;
  int record_timings = 0;
  int tile = 0;       // 0 = auto, else variant id + 1
  int order = ORDER_AUTO;
  int out_f32 = 0;    // C holds FP32 elements
  int patch_r = 4, patch_c = 8;  // C blocks per patch (ORDER_PATCH)
  int device_klists = 0;  // 0: when the triples would not fit the host list, 1: always, -1: never
  int trans_a = 0, trans_b = 0;  // the product reads A^T (B^T): the operand is stored transposed;
                                 // with complex elements 2 = the adjoint
  int cplx = 0;                  // complex elements (run as the real embedding)
  int k_split = 0;               // reduction variant: 0/1 off, n >= 2 pieces per k-list, -1 auto
  std::string tune_cache;  // autotuner choices file ("" = none)
};

// Size classes of C blocks (by the larger of the block's two sizes): <= 32, <= 64, <= 128, more.
// Each class has its own tile variant, so one plan or batch can mix variants.
constexpr int kSizeClasses = 4;
inline int size_class(int m, int n) {
  const int d = m > n ? m : n;
  return d <= 32 ? 0 : d <= 64 ? 1 : d <= 128 ? 2 : 3;
}

// A run of tasks that share one tile variant, launched together: tasks [begin, end) of the task
// list, dealt to the XCDs (tasks begin + xcd_begin[x] .. begin + xcd_begin[x+1] - 1 on XCD x).
struct Segment {
  int variant = 0;
  int32_t begin = 0, end = 0;
  int32_t xcd_begin[kXcds + 1] = {0};
  int64_t grid = 0;  // workgroups of the launch
  int64_t job_begin = 0, job_count = 0;  // device-built k-lists of the segment's C blocks
};

// Block triples the host list holds at most; beyond it (or on request) k-lists are built on the
// device, batch by batch, into a buffer of at most kDeviceTriples triples.
constexpr int64_t kHostTriples = int64_t(1) << 28;
constexpr int64_t kDeviceTriples = int64_t(1) << 27;

// A present C block and its k-list (the unit tasks are cut from).
struct CBlock {
  int64_t c_off;
  uint32_t tri_begin, tri_count;
  int32_t m, n;
  int32_t ci, cj;  // block row and column of C
  double sk;  // summed inner size of the k-list
};

// Host-side facts about a task the device does not need: its C block's position and its tile
// variant.
struct ItemMeta {
  int32_t ci, cj;
  int32_t var;
  double sk;  // summed inner size of the C block's k-list
};

struct HostPlan {
  PlanConfig cfg;
  int64_t M = 0, K = 0, N = 0;
  std::vector<int64_t> rows, inner, cols;
  std::vector<uint64_t> a_bits, b_bits, c_bits;  // shapes in the ABI word layout
  std::vector<int64_t> a_off, b_off, c_off;      // block offsets, -1 = absent
  int64_t a_blocks = 0, b_blocks = 0, c_blocks = 0;
  int64_t a_elems = 0, b_elems = 0, c_elems = 0;
  double useful_flops = 0.0;

  std::vector<Triple> tri;       // k-lists of all C blocks, C blocks in row-major order (host mode)
  // device-built k-lists: bitmaps, offset tables and the jobs of every segment
  bool dev_klists = false;
  int64_t wk = 0;                // 64-bit words per bitmap row of the inner dimension
  std::vector<uint64_t> bt_bits; // B's shape transposed: column j's k bits (N x wk)
  std::vector<int64_t> a_tab;    // M x K: packed offset of A_ik in the form's layout, -1 absent
  std::vector<int64_t> bt_tab;   // N x K: packed offset of B_kj at [j K + k], -1 absent
  std::vector<KJob> jobs;        // per segment (Segment::job_begin), C blocks of the segment
  int64_t tri_capacity = 0;      // triple buffer the device needs (largest segment)
  int64_t triples_total = 0;     // triples of the whole product
  std::vector<CBlock> cblocks;   // present C blocks, row-major
  double k_total = 0;            // summed inner size of all K blocks
  int class_var[kSizeClasses] = {0, 0, 0, 0};  // tile variant of each size class
  std::vector<Item> items;       // tasks in execution order: segment by segment, XCD by XCD
  std::vector<ItemMeta> meta;    // position and tile variant of items[q]
  std::vector<double> cost;      // scheduler cost of items[q]
  std::vector<float> features;   // 5 per item: log h, log w, log sum_k, log #k, density
  std::vector<Segment> segs;     // one per tile variant in use, in variant order
  // split-bf16 form: slice-plane layout of A and B and the split pass's block table
  int64_t a_elems32 = 0, b_elems32 = 0;
  std::vector<SplitBlock> split_a, split_b;
  // FP64 and FP32 forms with a transposed operand: the transposition pass's block tables (stored
  // blocks -> op(A), op(B) in the product's packed layout)
  std::vector<XposeBlock> xpose_a, xpose_b;
  // complex elements: this plan is the real embedding (rows and inner sizes doubled); the user's
  // view, the embedding pass's tables and the epilogue's C blocks
  int cplx = 0;
  int zop_a = 0, zop_b = 0;      // 0 as is, 1 transpose, 2 adjoint
  int z_out_f32 = 0;             // C holds complex FP32 elements
  std::vector<ZBlock> zembed_a, zembed_b;
  std::vector<ZCBlock> zc;
  // buffer sizes in the caller's elements (complex elements of a complex plan)
  int64_t user_a() const { return cplx ? a_elems / 4 : a_elems; }
  int64_t user_b() const { return cplx ? b_elems / 2 : b_elems; }
  int64_t user_c() const { return cplx ? c_elems / 2 : c_elems; }
  bool user_out_f32() const { return cplx ? z_out_f32 != 0 : cfg.out_f32 != 0; }
  int ksplit = 1;                // pieces each task's k-list is cut into (reduction variant)
  int64_t k_window_eff = 0;      // inner blocks per k-window
  int64_t windows = 1;           // number of k-windows

  // The tile variant every task uses, or -1 if the tasks mix variants.
  int uniform_variant() const {
    if (segs.empty()) return class_var[0];
    for (const Segment& g : segs)
      if (g.variant != segs[0].variant) return -1;
    return segs[0].variant;
  }
};

int64_t words_for(int64_t ncols);

// Returns "" on success, else an error text; *code receives the status.
std::string build_plan(HostPlan& p, int64_t M, const int64_t* rows, int64_t K,
                       const int64_t* inner, int64_t N, const int64_t* cols,
                       const uint64_t* a_bits, const uint64_t* b_bits, const PlanConfig& cfg,
                       int* code);

// Cut every C block into tasks with the tile variant of its size class (replaces items, meta and
// features; sets p.class_var).
void cut_items(HostPlan& p, const int class_var[kSizeClasses]);
// The same variant for every size class.
void cut_items(HostPlan& p, int variant);

// Re-order and re-partition the tasks from per-item costs (never changes the task set).
void schedule(HostPlan& p, const std::vector<double>& cost);

// Concatenate the tasks of several plans (same precision, one k-window) into one schedule; task q
// of part p keeps its triples and tile variant and is tagged with product p.
std::string merge_plans(HostPlan& out, const std::vector<const HostPlan*>& parts, int* code);

// Flop-count cost of every item.
std::vector<double> flop_costs(const HostPlan& p);

}  // namespace bsm
