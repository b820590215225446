// C ABI of the library (declared in include/bsm.h).
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/bsm.h"
#include "kernels.hpp"
#include "plan.hpp"

using namespace bsm;

static thread_local std::string g_error;

static bsm_status fail(bsm_status code, const std::string& msg) {
  g_error = msg;
  return code;
}

static bsm_status hip_fail(hipError_t e, const char* what) {
  return fail(BSM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

struct bsm_plan {
  HostPlan hp;
  Item* d_items = nullptr;
  Triple* d_tri = nullptr;
  void* d_opA = nullptr;         // converted operands of the reduced-precision forms
  void* d_opB = nullptr;
  SplitBlock* d_split_a = nullptr;  // split-bf16 form: block tables of the split pass
  SplitBlock* d_split_b = nullptr;
  double* d_partial = nullptr;   // raw sums between k-windows (laid out like C)
  uint64_t* d_stamps = nullptr;  // per-task start/end clocks
  int device = -1;
  bool uploaded = false;
  bool timed = false;            // an execute has recorded timings
};

extern "C" {

const char* bsm_last_error(void) { return g_error.c_str(); }

void bsm_options_default(bsm_options* opt) {
  if (!opt) return;
  opt->precision = BSM_FP64;
  opt->sched = BSM_SCHED_FLOPS;
  opt->k_window = 0;
  opt->record_timings = 0;
  opt->tile = 0;
}

int32_t bsm_tile_variants(int32_t* tm, int32_t* tn, int32_t cap) {
  for (int v = 0; v < kNumVariants && v < cap; ++v) {
    if (tm) tm[v] = kVariants[v].tm;
    if (tn) tn[v] = kVariants[v].tn;
  }
  return kNumVariants;
}

int64_t bsm_concurrent_iterations(int64_t p_row, int64_t p_col, int64_t K) {
  if (p_row < 2 || p_col < 2) return 2;
  if (p_row >= K && p_col >= K) return K;
  return p_row < p_col ? p_row : p_col;
}

bsm_status bsm_plan_create(bsm_plan** out, int64_t M, const int64_t* row_sizes, int64_t K,
                           const int64_t* inner_sizes, int64_t N, const int64_t* col_sizes,
                           const uint64_t* a_bits, const uint64_t* b_bits,
                           const bsm_options* opt) {
  if (!out) return fail(BSM_E_INVALID, "out is null");
  *out = nullptr;
  bsm_options o;
  bsm_options_default(&o);
  if (opt) o = *opt;
  PlanConfig cfg;
  cfg.precision = o.precision;
  cfg.sched = o.sched;
  cfg.k_window = o.k_window;
  cfg.record_timings = o.record_timings;
  cfg.tile = o.tile;
  if (const char* s = getenv("BSM_ORDER")) cfg.order = atoi(s);
  if (const char* s = getenv("BSM_CUT")) cfg.cut_search = atoi(s) != 0;
  bsm_plan* p = new (std::nothrow) bsm_plan;
  if (!p) return fail(BSM_E_NOMEM, "host allocation failed");
  int code = BSM_OK;
  std::string err;
  try {
    err = build_plan(p->hp, M, row_sizes, K, inner_sizes, N, col_sizes, a_bits, b_bits, cfg, &code);
  } catch (const std::bad_alloc&) {
    code = BSM_E_NOMEM;
    err = "host allocation failed while planning";
  }
  if (code != BSM_OK) {
    delete p;
    return fail(bsm_status(code), err);
  }
  *out = p;
  return BSM_OK;
}

bsm_status bsm_plan_query(const bsm_plan* plan, bsm_plan_info* info) {
  if (!plan || !info) return fail(BSM_E_INVALID, "null argument");
  const HostPlan& h = plan->hp;
  info->M = h.M;
  info->K = h.K;
  info->N = h.N;
  info->a_blocks = h.a_blocks;
  info->b_blocks = h.b_blocks;
  info->c_blocks = h.c_blocks;
  info->a_elems = h.a_elems;
  info->b_elems = h.b_elems;
  info->c_elems = h.c_elems;
  info->triples = int64_t(h.tri.size());
  info->tasks = int64_t(h.items.size());
  info->useful_flops = h.useful_flops;
  int64_t ws = int64_t(h.items.size() * sizeof(Item) + h.tri.size() * sizeof(Triple));
  if (h.cfg.precision == BSM_FP32) ws += (h.a_elems + h.b_elems) * 4;
  if (h.cfg.precision == BSM_BF16X3)
    ws += (h.a_elems32 + h.b_elems32) * 6 + int64_t((h.split_a.size() + h.split_b.size()) * sizeof(SplitBlock));
  if (h.windows > 1) ws += h.c_elems * 8;
  if (h.cfg.record_timings) ws += int64_t(h.items.size()) * 16;
  info->workspace_bytes = ws;
  info->k_windows = h.windows;
  return BSM_OK;
}

bsm_status bsm_plan_c_shape(const bsm_plan* plan, uint64_t* c_bits) {
  if (!plan || (!c_bits && !plan->hp.c_bits.empty())) return fail(BSM_E_INVALID, "null argument");
  if (!plan->hp.c_bits.empty())
    std::memcpy(c_bits, plan->hp.c_bits.data(), plan->hp.c_bits.size() * sizeof(uint64_t));
  return BSM_OK;
}

bsm_status bsm_plan_c_offsets(const bsm_plan* plan, int64_t* c_offsets) {
  if (!plan || (!c_offsets && !plan->hp.c_off.empty())) return fail(BSM_E_INVALID, "null argument");
  if (!plan->hp.c_off.empty())
    std::memcpy(c_offsets, plan->hp.c_off.data(), plan->hp.c_off.size() * sizeof(int64_t));
  return BSM_OK;
}

static bsm_status check_device(int* dev) {
  hipError_t e = hipGetDevice(dev);
  if (e != hipSuccess) return fail(BSM_E_UNSUPPORTED, std::string("no HIP device: ") + hipGetErrorString(e));
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, *dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(BSM_E_UNSUPPORTED, std::string("this library is built for gfx950, device is ") + prop.gcnArchName);
  return BSM_OK;
}

static bsm_status upload(bsm_plan* p) {
  if (p->uploaded) return BSM_OK;
  int dev;
  bsm_status st = check_device(&dev);
  if (st != BSM_OK) return st;
  const HostPlan& h = p->hp;
  hipError_t e;
  if (!h.items.empty()) {
    if ((e = hipMalloc(&p->d_items, h.items.size() * sizeof(Item))) != hipSuccess) return hip_fail(e, "hipMalloc(tasks)");
    if ((e = hipMemcpy(p->d_items, h.items.data(), h.items.size() * sizeof(Item), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "hipMemcpy(tasks)");
  }
  if (!h.tri.empty()) {
    if ((e = hipMalloc(&p->d_tri, h.tri.size() * sizeof(Triple))) != hipSuccess) return hip_fail(e, "hipMalloc(triples)");
    if ((e = hipMemcpy(p->d_tri, h.tri.data(), h.tri.size() * sizeof(Triple), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "hipMemcpy(triples)");
  }
  const int64_t ne_a = h.a_elems, ne_b = h.b_elems;
  if (h.cfg.precision == BSM_FP32) {
    if (ne_a > 0 && (e = hipMalloc(&p->d_opA, size_t(ne_a) * 4)) != hipSuccess) return hip_fail(e, "hipMalloc(A fp32)");
    if (ne_b > 0 && (e = hipMalloc(&p->d_opB, size_t(ne_b) * 4)) != hipSuccess) return hip_fail(e, "hipMalloc(B fp32)");
  }
  if (h.cfg.precision == BSM_BF16X3) {
    if (h.a_elems32 > 0 && (e = hipMalloc(&p->d_opA, size_t(h.a_elems32) * 6)) != hipSuccess) return hip_fail(e, "hipMalloc(A slices)");
    if (h.b_elems32 > 0 && (e = hipMalloc(&p->d_opB, size_t(h.b_elems32) * 6)) != hipSuccess) return hip_fail(e, "hipMalloc(B slices)");
    const size_t na = h.split_a.size() * sizeof(SplitBlock), nb = h.split_b.size() * sizeof(SplitBlock);
    if (na && (e = hipMalloc(&p->d_split_a, na)) != hipSuccess) return hip_fail(e, "hipMalloc(split table)");
    if (nb && (e = hipMalloc(&p->d_split_b, nb)) != hipSuccess) return hip_fail(e, "hipMalloc(split table)");
    if (na && (e = hipMemcpy(p->d_split_a, h.split_a.data(), na, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy(split table)");
    if (nb && (e = hipMemcpy(p->d_split_b, h.split_b.data(), nb, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e, "hipMemcpy(split table)");
  }
  if (h.windows > 1 && h.c_elems > 0) {
    if ((e = hipMalloc(&p->d_partial, size_t(h.c_elems) * 8)) != hipSuccess) return hip_fail(e, "hipMalloc(partial)");
  }
  if (h.cfg.record_timings && !h.items.empty()) {
    if ((e = hipMalloc(&p->d_stamps, h.items.size() * 16)) != hipSuccess) return hip_fail(e, "hipMalloc(stamps)");
  }
  p->device = dev;
  p->uploaded = true;
  return BSM_OK;
}

static bool overlaps(const void* a, int64_t na, const void* b, int64_t nb) {
  if (na <= 0 || nb <= 0) return false;
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

bsm_status bsm_execute(bsm_plan* plan, double alpha, const double* dA, const double* dB,
                       double* dC, int accumulate, void* stream) {
  if (!plan) return fail(BSM_E_INVALID, "plan is null");
  const HostPlan& h = plan->hp;
  if ((h.a_elems > 0 && !dA) || (h.b_elems > 0 && !dB) || (h.c_elems > 0 && !dC))
    return fail(BSM_E_INVALID, "null tile buffer");
  if (overlaps(dC, h.c_elems * 8, dA, h.a_elems * 8) || overlaps(dC, h.c_elems * 8, dB, h.b_elems * 8))
    return fail(BSM_E_INVALID, "C overlaps A or B");
  if (accumulate != 0 && accumulate != 1) return fail(BSM_E_INVALID, "accumulate must be 0 or 1");
  bsm_status st = upload(plan);
  if (st != BSM_OK) return st;
  if (h.items.empty()) return BSM_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  int form = FORM_F64;
  const void* opA = dA;
  const void* opB = dB;
  if (h.cfg.precision == BSM_FP32) {
    // S6: operands rounded to FP32 once per execute (A == B is converted once)
    form = FORM_F32;
    if ((e = launch_to_f32(dA, static_cast<float*>(plan->d_opA), h.a_elems, s)) != hipSuccess)
      return hip_fail(e, "convert A");
    opA = plan->d_opA;
    if (dB == dA && h.b_elems == h.a_elems) {
      opB = plan->d_opA;
    } else {
      if ((e = launch_to_f32(dB, static_cast<float*>(plan->d_opB), h.b_elems, s)) != hipSuccess)
        return hip_fail(e, "convert B");
      opB = plan->d_opB;
    }
  }
  int64_t a_plane = 0, b_plane = 0;
  if (h.cfg.precision == BSM_BF16X3) {
    // S6: three bf16 slices of every operand element, inner size padded to 32, B transposed
    form = FORM_BF16X3;
    a_plane = h.a_elems32;
    b_plane = h.b_elems32;
    if ((e = launch_split_bf16x3(plan->d_split_a, int64_t(h.split_a.size()), dA,
                                 static_cast<uint16_t*>(plan->d_opA), a_plane, s)) != hipSuccess)
      return hip_fail(e, "split A");
    if ((e = launch_split_bf16x3(plan->d_split_b, int64_t(h.split_b.size()), dB,
                                 static_cast<uint16_t*>(plan->d_opB), b_plane, s)) != hipSuccess)
      return hip_fail(e, "split B");
    opA = plan->d_opA;
    opB = plan->d_opB;
  }
  TileArgs a{};
  a.items = plan->d_items;
  a.tri = plan->d_tri;
  for (int x = 0; x <= kXcds; ++x) a.map.begin[x] = h.xcd_begin[x];
  a.prods = nullptr;
  a.single = ProductArgs{opA, opB, dC, plan->d_partial, alpha, a_plane, b_plane};
  a.accumulate = accumulate;
  a.stamps = plan->d_stamps;
  // S5: k-windows of I consecutive inner blocks, issued in order on the stream; each window
  // resumes from the raw FP64 sums of the previous one, so C does not depend on I
  const int64_t I = h.k_window_eff;
  for (int64_t wdx = 0; wdx < h.windows; ++wdx) {
    a.k_lo = int(wdx * I);
    a.k_hi = wdx + 1 == h.windows ? kNoKLimit : int((wdx + 1) * I);
    a.win_first = wdx == 0;
    a.win_last = wdx + 1 == h.windows;
    const int v = h.items[0].variant;
    e = form == FORM_F64   ? launch_tiles_f64(v, h.grid, a, s)
        : form == FORM_F32 ? launch_tiles_f32(v, h.grid, a, s)
                           : launch_tiles_bf16x3(v, h.grid, a, s);
    if (e != hipSuccess) return hip_fail(e, "tile kernel launch");
  }
  plan->timed = plan->d_stamps != nullptr;
  return BSM_OK;
}

bsm_status bsm_plan_timings(bsm_plan* plan, float* features, float* seconds, int64_t n,
                            void* stream) {
  if (!plan) return fail(BSM_E_INVALID, "plan is null");
  const HostPlan& h = plan->hp;
  if (n != int64_t(h.items.size())) return fail(BSM_E_MISMATCH, "n must equal the task count");
  if (!plan->timed) return fail(BSM_E_STATE, "no execute with record_timings has run");
  if (n == 0) return BSM_OK;
  if ((!features && !seconds)) return fail(BSM_E_INVALID, "null output");
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  std::vector<uint64_t> st(size_t(n) * 2);
  e = hipMemcpy(st.data(), plan->d_stamps, st.size() * 8, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(stamps)");
  for (int64_t q = 0; q < n; ++q) {
    if (seconds) seconds[q] = float(double(st[size_t(2 * q + 1)] - st[size_t(2 * q)]) * 1e-8);
    if (features)
      for (int f = 0; f < 5; ++f) features[q * 5 + f] = h.features[size_t(q * 5 + f)];
  }
  return BSM_OK;
}

bsm_status bsm_plan_destroy(bsm_plan* plan) {
  if (!plan) return BSM_OK;
  bsm_status st = BSM_OK;
  if (plan->uploaded) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) st = hip_fail(e, "hipDeviceSynchronize");
    for (void* ptr : {static_cast<void*>(plan->d_items), static_cast<void*>(plan->d_tri), plan->d_opA,
                      plan->d_opB, static_cast<void*>(plan->d_split_a), static_cast<void*>(plan->d_split_b),
                      static_cast<void*>(plan->d_partial), static_cast<void*>(plan->d_stamps)})
      if (ptr) (void)hipFree(ptr);
  }
  delete plan;
  return st;
}

}  // extern "C"
