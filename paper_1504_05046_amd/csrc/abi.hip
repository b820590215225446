// C ABI of the library (declared in include/bsm.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/bsm.h"
#include "errors.hpp"
#include "kernels.hpp"
#include "plan.hpp"

using namespace bsm;

static thread_local std::string g_error;

static bsm_status fail(bsm_status code, const std::string& msg) {
  g_error = msg;
  return code;
}

bsm_status bsm::set_error(bsm_status code, const std::string& msg) { return fail(code, msg); }

static bsm_status hip_fail(hipError_t e, const char* what) {
  return fail(BSM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define BSM_HIP(call, what)                          \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// ------------------------------------------------------------------------------------------------
// Device copies of a task list: tasks, triples, per-task execution counters, optional per-task
// clocks.
struct TaskSet {
  Item* items = nullptr;
  Triple* tri = nullptr;     // the host list, or the buffer device-built k-lists go into
  KJob* jobs = nullptr;      // device-built k-lists: the C blocks of every segment
  size_t n_jobs = 0;
  uint64_t* stamps = nullptr;
  uint32_t* done = nullptr;  // executions of each task since the last upload
  size_t n_items = 0, n_tri = 0;
  int64_t expected = 0;      // executions every task should have had by now
  bool timed = false;        // a launch has recorded clocks since the tasks last changed
  bool used = false;         // work that reads these buffers may be queued

  void release() {
    for (void* ptr : {static_cast<void*>(items), static_cast<void*>(tri), static_cast<void*>(jobs),
                      static_cast<void*>(stamps), static_cast<void*>(done)})
      if (ptr) (void)hipFree(ptr);
    items = nullptr;
    tri = nullptr;
    jobs = nullptr;
    stamps = nullptr;
    done = nullptr;
    n_items = n_tri = n_jobs = 0;
  }

  // (Re-)upload tasks (always) and triples (when their count changed); clocks if asked for.
  // Launches queued earlier on `stream` may still read the old tables, so they are waited for
  // first.  The execution counters start again from zero.
  bsm_status upload(const HostPlan& h, bool with_stamps, hipStream_t stream) {
    if (used) BSM_HIP(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (h.items.size() != n_items) {
      for (void* ptr : {static_cast<void*>(items), static_cast<void*>(stamps), static_cast<void*>(done)})
        if (ptr) (void)hipFree(ptr);
      items = nullptr;
      stamps = nullptr;
      done = nullptr;
      n_items = h.items.size();
      if (n_items) BSM_HIP(hipMalloc(&items, n_items * sizeof(Item)), "hipMalloc(tasks)");
      if (n_items) BSM_HIP(hipMalloc(&done, n_items * sizeof(uint32_t)), "hipMalloc(counters)");
    }
    if (n_items) BSM_HIP(hipMemset(done, 0, n_items * sizeof(uint32_t)), "hipMemset(counters)");
    expected = 0;
    if (n_items)
      BSM_HIP(hipMemcpy(items, h.items.data(), n_items * sizeof(Item), hipMemcpyHostToDevice),
              "hipMemcpy(tasks)");
    const size_t want_tri = h.dev_klists ? size_t(h.tri_capacity) : h.tri.size();
    if (want_tri != n_tri) {
      if (tri) (void)hipFree(tri);
      tri = nullptr;
      n_tri = want_tri;
      if (n_tri) BSM_HIP(hipMalloc(&tri, n_tri * sizeof(Triple)), "hipMalloc(triples)");
    }
    if (n_tri && !h.dev_klists)
      BSM_HIP(hipMemcpy(tri, h.tri.data(), n_tri * sizeof(Triple), hipMemcpyHostToDevice),
              "hipMemcpy(triples)");
    if (h.jobs.size() != n_jobs) {
      if (jobs) (void)hipFree(jobs);
      jobs = nullptr;
      n_jobs = h.jobs.size();
      if (n_jobs) BSM_HIP(hipMalloc(&jobs, n_jobs * sizeof(KJob)), "hipMalloc(k-list jobs)");
    }
    if (n_jobs)
      BSM_HIP(hipMemcpy(jobs, h.jobs.data(), n_jobs * sizeof(KJob), hipMemcpyHostToDevice),
              "hipMemcpy(k-list jobs)");
    if (with_stamps && !stamps && n_items)
      BSM_HIP(hipMalloc(&stamps, n_items * 16), "hipMalloc(clocks)");
    timed = false;
    return BSM_OK;
  }

  // Waits for `stream`, then checks that every task ran exactly `expected` times.
  bsm_status verify(hipStream_t stream) {
    BSM_HIP(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (!n_items) return BSM_OK;
    std::vector<uint32_t> c(n_items);
    BSM_HIP(hipMemcpy(c.data(), done, n_items * sizeof(uint32_t), hipMemcpyDeviceToHost),
            "hipMemcpy(counters)");
    for (size_t q = 0; q < n_items; ++q)
      if (int64_t(c[q]) != expected) {
        g_error = "task " + std::to_string(q) + " ran " + std::to_string(c[q]) +
                  " times, expected " + std::to_string(expected);
        return BSM_E_STATE;
      }
    return BSM_OK;
  }
};

// A captured launch sequence, replayed while its arguments stay the same.  Capture happens on a
// private stream; the instantiated graph is launched on the caller's stream.
struct GraphCache {
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<uint64_t> key;
  bool valid = false;

  void invalidate() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    valid = false;
  }
  void release() {
    invalidate();
    if (cap) (void)hipStreamDestroy(cap);
    cap = nullptr;
  }
  bsm_status run(const std::vector<uint64_t>& k, const std::function<bsm_status(hipStream_t)>& body,
                 hipStream_t stream) {
    if (!valid || k != key) {
      invalidate();
      if (!cap) BSM_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "hipStreamCreate");
      BSM_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
      bsm_status st = body(cap);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(cap, &g);
      if (st != BSM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
      graph = g;
      BSM_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
      key = k;
      valid = true;
    }
    BSM_HIP(hipGraphLaunch(exec, stream), "hipGraphLaunch");
    return BSM_OK;
  }
};

static uint64_t bits_of(double d) {
  uint64_t u;
  std::memcpy(&u, &d, 8);
  return u;
}

// ------------------------------------------------------------------------------------------------
// Operands as the tile kernels read them when not in place (staged_bytes > 0): the buffers and
// the block tables of the passes that fill them.
struct Staging {
  void* opA = nullptr;
  void* opB = nullptr;
  const SplitBlock* sa = nullptr;  // split-bf16 form: block tables of the split pass
  const SplitBlock* sb = nullptr;
  const XposeBlock* xa = nullptr;  // transposed operands: block tables of the transposition pass
  const XposeBlock* xb = nullptr;
};

// Bytes of the staged copy of A (or B): the FP32 copy, the bf16 slice planes, or op(X) of a
// transposed FP64 operand; 0 = the tile kernels read the caller's buffer.
static int64_t staged_bytes(const HostPlan& h, bool b) {
  switch (h.cfg.precision) {
    case BSM_FP32: return (b ? h.b_elems : h.a_elems) * 4;
    case BSM_BF16X3: return (b ? h.b_elems32 : h.a_elems32) * 6;
    default: return (b ? h.cfg.trans_b : h.cfg.trans_a) ? (b ? h.b_elems : h.a_elems) * 8 : 0;
  }
}

// Bytes of the block tables of the staging passes.
static int64_t staging_table_bytes(const HostPlan& h) {
  return int64_t((h.split_a.size() + h.split_b.size()) * sizeof(SplitBlock) +
                 (h.xpose_a.size() + h.xpose_b.size()) * sizeof(XposeBlock) +
                 (h.zembed_a.size() + h.zembed_b.size()) * sizeof(ZBlock) +
                 h.zc.size() * sizeof(ZCBlock));
}

// Complex elements: bytes of the embedded operands and of the real product's C.
static int64_t complex_bytes(const HostPlan& h) {
  return h.cplx ? (h.a_elems + h.b_elems + h.c_elems) * 8 : 0;
}

struct bsm_plan {
  HostPlan hp;
  TaskSet ts;
  void* d_opA = nullptr;            // staged operands (staged_bytes)
  void* d_opB = nullptr;
  SplitBlock* d_split_a = nullptr;  // split-bf16 form: block tables of the split pass
  SplitBlock* d_split_b = nullptr;
  XposeBlock* d_xpose_a = nullptr;  // transposed operands: block tables of the transposition pass
  XposeBlock* d_xpose_b = nullptr;
  double* d_zA = nullptr;           // complex elements: the embedded operands, the real product's
  double* d_zB = nullptr;           // [Re; Im] C blocks, and the tables of the passes
  double* d_zP = nullptr;
  ZBlock* d_zembed_a = nullptr;
  ZBlock* d_zembed_b = nullptr;
  ZCBlock* d_zc = nullptr;
  double* d_splitP = nullptr;       // reduction variant: ksplit partial sums laid out like C
  ProductArgs* d_kprods = nullptr;  // ... and the operand table of the pieces
  std::vector<ProductArgs> h_kprods;
  bool kprods_used = false;         // a queued launch may read d_kprods
  double* d_partial = nullptr;      // raw sums between k-windows (laid out like C)
  // device-built k-lists: shapes, offset tables and inner sizes
  uint64_t* d_abits = nullptr;
  uint64_t* d_btbits = nullptr;
  int64_t* d_atab = nullptr;
  int64_t* d_bttab = nullptr;
  int64_t* d_inner = nullptr;
  DevKlists dk{};
  GraphCache gc;
  int device = -1;
  bool ready = false;               // device buffers allocated
  bool tasks_dirty = true;          // host tasks changed since the last upload
  int use_graph = 0;
  int skip_task = -1;               // fault injection: task left out of every launch
};

struct bsm_batch {
  std::vector<bsm_plan*> members;
  HostPlan hp;                      // merged tasks
  TaskSet ts;
  ProductArgs* d_prods = nullptr;
  std::vector<ProductArgs> h_prods;
  GraphCache gc;
  bool tasks_dirty = true;
  bool table_used = false;          // a queued launch may read d_prods
};

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

// Device buffers of a plan other than its task list.
// Every device buffer of a plan besides its task list (freed by release_buffers).
static std::vector<void**> buffer_slots(bsm_plan* p) {
  return {&p->d_opA, &p->d_opB,
          reinterpret_cast<void**>(&p->d_split_a), reinterpret_cast<void**>(&p->d_split_b),
          reinterpret_cast<void**>(&p->d_xpose_a), reinterpret_cast<void**>(&p->d_xpose_b),
          reinterpret_cast<void**>(&p->d_partial), reinterpret_cast<void**>(&p->d_zA),
          reinterpret_cast<void**>(&p->d_zB), reinterpret_cast<void**>(&p->d_zP),
          reinterpret_cast<void**>(&p->d_zembed_a), reinterpret_cast<void**>(&p->d_zembed_b),
          reinterpret_cast<void**>(&p->d_zc), reinterpret_cast<void**>(&p->d_splitP),
          reinterpret_cast<void**>(&p->d_kprods), reinterpret_cast<void**>(&p->d_abits),
          reinterpret_cast<void**>(&p->d_btbits), reinterpret_cast<void**>(&p->d_atab),
          reinterpret_cast<void**>(&p->d_bttab), reinterpret_cast<void**>(&p->d_inner)};
}

// Frees every buffer of buffer_slots (after the device is idle) and clears the pointers.
static bsm_status release_buffers(bsm_plan* p) {
  bool any = false;
  for (void** s : buffer_slots(p)) any = any || *s;
  if (!any) return BSM_OK;
  hipError_t e = hipDeviceSynchronize();
  for (void** s : buffer_slots(p)) {
    if (*s) (void)hipFree(*s);
    *s = nullptr;
  }
  p->h_kprods.clear();
  p->dk = DevKlists{};
  return e == hipSuccess ? BSM_OK : hip_fail(e, "hipDeviceSynchronize");
}

static bsm_status prepare_buffers(bsm_plan* p);

// Device buffers of a plan other than its task list; a failure part-way releases what was
// allocated, so that a later call starts again from nothing.
static bsm_status prepare(bsm_plan* p) {
  if (p->ready) return BSM_OK;
  const bsm_status st = prepare_buffers(p);
  if (st != BSM_OK) {
    const std::string msg = g_error;
    (void)release_buffers(p);
    return fail(st, msg);
  }
  return BSM_OK;
}

static bsm_status prepare_buffers(bsm_plan* p) {
  int dev;
  bsm_status st = check_device(&dev);
  if (st != BSM_OK) return st;
  const HostPlan& h = p->hp;
  const int64_t sa = staged_bytes(h, false), sb = staged_bytes(h, true);
  if (sa > 0) BSM_HIP(hipMalloc(&p->d_opA, size_t(sa)), "hipMalloc(staged A)");
  if (sb > 0) BSM_HIP(hipMalloc(&p->d_opB, size_t(sb)), "hipMalloc(staged B)");
  auto table = [&](auto** dst, const auto& v) -> bsm_status {
    const size_t bytes = v.size() * sizeof(v[0]);
    if (!bytes) return BSM_OK;
    BSM_HIP(hipMalloc(dst, bytes), "hipMalloc(staging table)");
    BSM_HIP(hipMemcpy(*dst, v.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy(staging table)");
    return BSM_OK;
  };
  bsm_status s1;
  if ((s1 = table(&p->d_split_a, h.split_a)) != BSM_OK) return s1;
  if ((s1 = table(&p->d_split_b, h.split_b)) != BSM_OK) return s1;
  if ((s1 = table(&p->d_xpose_a, h.xpose_a)) != BSM_OK) return s1;
  if ((s1 = table(&p->d_xpose_b, h.xpose_b)) != BSM_OK) return s1;
  if (h.cplx) {
    if ((s1 = table(&p->d_zembed_a, h.zembed_a)) != BSM_OK) return s1;
    if ((s1 = table(&p->d_zembed_b, h.zembed_b)) != BSM_OK) return s1;
    if ((s1 = table(&p->d_zc, h.zc)) != BSM_OK) return s1;
    if (h.a_elems > 0) BSM_HIP(hipMalloc(&p->d_zA, size_t(h.a_elems) * 8), "hipMalloc(embedded A)");
    if (h.b_elems > 0) BSM_HIP(hipMalloc(&p->d_zB, size_t(h.b_elems) * 8), "hipMalloc(embedded B)");
    if (h.c_elems > 0) BSM_HIP(hipMalloc(&p->d_zP, size_t(h.c_elems) * 8), "hipMalloc(complex C parts)");
  }
  if (h.ksplit > 1) {
    if (h.c_elems > 0)
      BSM_HIP(hipMalloc(&p->d_splitP, size_t(h.c_elems) * 8 * size_t(h.ksplit)), "hipMalloc(partial sums)");
    BSM_HIP(hipMalloc(&p->d_kprods, sizeof(ProductArgs) * size_t(h.ksplit)), "hipMalloc(piece table)");
  }
  if (h.windows > 1 && h.c_elems > 0)
    BSM_HIP(hipMalloc(&p->d_partial, size_t(h.c_elems) * 8), "hipMalloc(partial)");
  if (h.dev_klists) {
    auto up = [&](auto** dst, const auto& v, const char* what) -> bsm_status {
      const size_t bytes = v.size() * sizeof(v[0]);
      if (!bytes) return BSM_OK;
      BSM_HIP(hipMalloc(dst, bytes), what);
      BSM_HIP(hipMemcpy(*dst, v.data(), bytes, hipMemcpyHostToDevice), what);
      return BSM_OK;
    };
    bsm_status s2;
    if ((s2 = up(&p->d_abits, h.a_bits, "k-list tables")) != BSM_OK) return s2;
    if ((s2 = up(&p->d_btbits, h.bt_bits, "k-list tables")) != BSM_OK) return s2;
    if ((s2 = up(&p->d_atab, h.a_tab, "k-list tables")) != BSM_OK) return s2;
    if ((s2 = up(&p->d_bttab, h.bt_tab, "k-list tables")) != BSM_OK) return s2;
    if ((s2 = up(&p->d_inner, h.inner, "k-list tables")) != BSM_OK) return s2;
    p->dk = DevKlists{p->d_abits, p->d_btbits, h.wk, p->d_atab, p->d_bttab, h.K, p->d_inner};
  }
  p->device = dev;
  p->ready = true;
  return BSM_OK;
}

static bsm_status sync_tasks(bsm_plan* p, hipStream_t stream) {
  if (!p->tasks_dirty) return BSM_OK;
  bsm_status st = p->ts.upload(p->hp, p->hp.cfg.record_timings != 0, stream);
  if (st != BSM_OK) return st;
  p->tasks_dirty = false;
  p->gc.invalidate();
  return BSM_OK;
}

// C = A A in the FP32 form with neither operand transposed: one FP32 copy serves both.
static bool shares_f32_copy(const HostPlan& h, const double* dA, const double* dB) {
  return h.cfg.precision == BSM_FP32 && !h.cfg.trans_a && !h.cfg.trans_b && dB == dA &&
         h.b_elems == h.a_elems;
}

// Where the tile kernels read op(A) and op(B): the caller's buffers or the staged copies.
static void bind_operands(const HostPlan& h, const double* dA, const double* dB, const Staging& g,
                          ProductArgs& pa) {
  pa.A = staged_bytes(h, false) > 0 ? g.opA : dA;
  pa.B = staged_bytes(h, true) > 0 ? (shares_f32_copy(h, dA, dB) ? g.opA : g.opB) : dB;
  pa.a_plane = h.cfg.precision == BSM_BF16X3 ? h.a_elems32 : 0;
  pa.b_plane = h.cfg.precision == BSM_BF16X3 ? h.b_elems32 : 0;
}

// S6: operands in the precision form's element type and the product's layout (queued on s),
// written into the staged copies: FP32 copies (transposed block by block for a transposed
// operand), bf16 slice planes built with the split tables, or op(X) of a transposed FP64 operand.
static bsm_status convert_into(const HostPlan& h, const double* dA, const double* dB,
                               const Staging& g, hipStream_t s, ProductArgs& pa) {
  bind_operands(h, dA, dB, g, pa);
  const bool ta = h.cfg.trans_a != 0, tb = h.cfg.trans_b != 0;
  if (h.cfg.precision == BSM_FP32) {
    if (ta)
      BSM_HIP(launch_transpose_f32(g.xa, int64_t(h.xpose_a.size()), dA, static_cast<float*>(g.opA), s),
              "transpose A");
    else
      BSM_HIP(launch_to_f32(dA, static_cast<float*>(g.opA), h.a_elems, s), "convert A");
    if (shares_f32_copy(h, dA, dB)) return BSM_OK;
    if (tb)
      BSM_HIP(launch_transpose_f32(g.xb, int64_t(h.xpose_b.size()), dB, static_cast<float*>(g.opB), s),
              "transpose B");
    else
      BSM_HIP(launch_to_f32(dB, static_cast<float*>(g.opB), h.b_elems, s), "convert B");
  } else if (h.cfg.precision == BSM_BF16X3) {
    BSM_HIP(launch_split_bf16x3(g.sa, int64_t(h.split_a.size()), dA, static_cast<uint16_t*>(g.opA),
                                pa.a_plane, s), "split A");
    BSM_HIP(launch_split_bf16x3(g.sb, int64_t(h.split_b.size()), dB, static_cast<uint16_t*>(g.opB),
                                pa.b_plane, s), "split B");
  } else {
    if (ta)
      BSM_HIP(launch_transpose_f64(g.xa, int64_t(h.xpose_a.size()), dA, static_cast<double*>(g.opA), s),
              "transpose A");
    if (tb)
      BSM_HIP(launch_transpose_f64(g.xb, int64_t(h.xpose_b.size()), dB, static_cast<double*>(g.opB), s),
              "transpose B");
  }
  return BSM_OK;
}

static Staging staging_of(const bsm_plan* p) {
  return Staging{p->d_opA, p->d_opB, p->d_split_a, p->d_split_b, p->d_xpose_a, p->d_xpose_b};
}

static bsm_status enqueue_convert(bsm_plan* p, const double* dA, const double* dB, hipStream_t s,
                                  ProductArgs& pa) {
  return convert_into(p->hp, dA, dB, staging_of(p), s, pa);
}

// The whole product on stream q: (complex: embedding of the operands), operand staging, the tile
// launches, (complex: the epilogue with alpha = ar + i ai).  Real plans take alpha = ar.
static bsm_status enqueue_product(bsm_plan* plan, double ar, double ai, const double* dA,
                                  const double* dB, void* dC, int accumulate, int skip,
                                  hipStream_t q);

static hipError_t launch_form(int precision, int variant, int64_t grid, const TileArgs& a,
                              hipStream_t s) {
  if (precision == BSM_FP64) return launch_tiles_f64(variant, grid, a, s);
  if (precision == BSM_FP32) return launch_tiles_f32(variant, grid, a, s);
  return launch_tiles_bf16x3(variant, grid, a, s);
}

// S7/S8 (and S5): the tile kernel over a task list, once per k-window.
static bsm_status enqueue_tiles(const HostPlan& h, TaskSet& ts, const ProductArgs* prods,
                                const ProductArgs& single, int accumulate, int skip_task,
                                hipStream_t s, const DevKlists* dk = nullptr) {
  if (h.items.empty()) return BSM_OK;
  // k-windows of I consecutive inner blocks, issued in order on the stream; each window resumes
  // from the raw FP64 sums of the previous one, so C does not depend on I.  Within a window, one
  // launch per segment (the tasks of one tile variant).
  const int64_t I = h.k_window_eff;
  for (int64_t wdx = 0; wdx < h.windows; ++wdx) {
    for (const Segment& g : h.segs) {
      if (h.dev_klists) {
        // this batch's k-lists into the triple buffer (after the previous batch's tiles)
        if (!dk) return fail(BSM_E_STATE, "device k-lists without their tables");
        BSM_HIP(launch_fill_klists(ts.jobs + g.job_begin, g.job_count, *dk, ts.tri, s), "k-list fill");
      }
      TileArgs a{};
      a.items = ts.items + g.begin;
      a.tri = ts.tri;
      a.done = ts.done ? ts.done + g.begin : nullptr;
      a.stamps = ts.stamps ? ts.stamps + 2 * int64_t(g.begin) : nullptr;
      a.skip_task = (skip_task >= g.begin && skip_task < g.end) ? skip_task - g.begin : -1;
      for (int x = 0; x <= kXcds; ++x) a.map.begin[x] = g.xcd_begin[x];
      a.prods = prods;
      a.single = single;
      a.accumulate = accumulate;
      a.k_lo = int(wdx * I);
      a.k_hi = wdx + 1 == h.windows ? kNoKLimit : int((wdx + 1) * I);
      a.win_first = wdx == 0;
      a.win_last = wdx + 1 == h.windows;
      BSM_HIP(launch_form(h.cfg.precision, g.variant, g.grid, a, s), "tile kernel launch");
    }
  }
  if (ts.stamps) ts.timed = true;
  return BSM_OK;
}

static bool overlaps(const void* a, int64_t na, const void* b, int64_t nb) {
  if (na <= 0 || nb <= 0) return false;
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

static bsm_status check_operands(const HostPlan& h, const double* dA, const double* dB,
                                 const void* dC, int accumulate) {
  if ((h.a_elems > 0 && !dA) || (h.b_elems > 0 && !dB) || (h.c_elems > 0 && !dC))
    return fail(BSM_E_INVALID, "null tile buffer");
  const int64_t es = h.cplx ? 16 : 8;  // bytes per element of A and B
  const int64_t cb = h.user_c() * (h.user_out_f32() ? 4 : 8) * (h.cplx ? 2 : 1);
  if (overlaps(dC, cb, dA, h.user_a() * es) || overlaps(dC, cb, dB, h.user_b() * es))
    return fail(BSM_E_INVALID, "C overlaps A or B");
  if (h.cplx && ((uintptr_t(dA) | uintptr_t(dB)) % 16 || uintptr_t(dC) % (h.user_out_f32() ? 8 : 16)))
    return fail(BSM_E_INVALID, "complex buffers must be aligned to their element size");
  if (accumulate != 0 && accumulate != 1) return fail(BSM_E_INVALID, "accumulate must be 0 or 1");
  return BSM_OK;
}

static bsm_status timings_of(const HostPlan& h, TaskSet& ts, float* features, float* seconds,
                             int64_t n, void* stream) {
  if (n != int64_t(h.items.size())) return fail(BSM_E_MISMATCH, "n must equal the task count");
  if (!ts.timed) return fail(BSM_E_STATE, "no execute with record_timings has run since the tasks last changed");
  if (n == 0) return BSM_OK;
  if (!features && !seconds) return fail(BSM_E_INVALID, "null output");
  bsm_status vs = ts.verify(static_cast<hipStream_t>(stream));  // synchronises the stream
  if (vs != BSM_OK) return vs;
  std::vector<uint64_t> st(size_t(n) * 2);
  BSM_HIP(hipMemcpy(st.data(), ts.stamps, st.size() * 8, hipMemcpyDeviceToHost), "hipMemcpy(clocks)");
  for (int64_t q = 0; q < n; ++q) {
    // the constant clock runs at 100 MHz
    if (seconds) seconds[q] = float(double(st[size_t(2 * q + 1)] - st[size_t(2 * q)]) * 1e-8);
    if (features)
      for (int f = 0; f < 5; ++f) features[q * 5 + f] = h.features[size_t(q * 5 + f)];
  }
  return BSM_OK;
}

static bsm_status set_costs(HostPlan& h, const float* costs, int64_t n) {
  if (n != int64_t(h.items.size())) return fail(BSM_E_MISMATCH, "n must equal the task count");
  if (n > 0 && !costs) return fail(BSM_E_INVALID, "null costs");
  std::vector<double> c(static_cast<size_t>(n));
  for (int64_t q = 0; q < n; ++q) {
    if (!(costs[q] >= 0.f) || !std::isfinite(costs[q])) return fail(BSM_E_INVALID, "costs must be finite and >= 0");
    c[size_t(q)] = costs[q];
  }
  schedule(h, c);
  return BSM_OK;
}

// ------------------------------------------------------------------------------------------------
// Autotuning: time each tile variant on the caller's operands and keep the fastest.  Choices are
// remembered per workload signature in the plan's tune-cache file (lines "key variant").
static std::string tune_key(const std::vector<const HostPlan*>& parts) {
  double nb = 0, sm = 0, sn = 0, sk = 0;
  for (const HostPlan* p : parts)
    for (const CBlock& c : p->cblocks) {
      nb += 1;
      sm += c.m;
      sn += c.n;
      sk += c.sk;
    }
  char buf[160];
  std::snprintf(buf, sizeof buf, "gfx950/p%d/b%zu/c%.0f/m%.0f/n%.0f/k%.0f", parts[0]->cfg.precision,
                parts.size(), nb, nb > 0 ? sm / nb : 0, nb > 0 ? sn / nb : 0, nb > 0 ? sk / nb : 0);
  return buf;
}

// A cache line holds the key and the variant of each size class ("key v0,v1,v2,v3"); the last
// line for a key wins.  Returns false if the key is absent or a variant is out of range.
static bool tune_cache_lookup(const std::string& path, const std::string& key, int nvar,
                              int cv[kSizeClasses]) {
  if (path.empty()) return false;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  char k[256];
  int v[kSizeClasses];
  bool found = false;
  while (std::fscanf(f, "%255s %d,%d,%d,%d", k, &v[0], &v[1], &v[2], &v[3]) == 5) {
    if (key != k) continue;
    bool ok = true;
    for (int c = 0; c < kSizeClasses; ++c) ok = ok && v[c] >= 0 && v[c] < nvar;
    if (!ok) continue;
    for (int c = 0; c < kSizeClasses; ++c) cv[c] = v[c];
    found = true;
  }
  std::fclose(f);
  return found;
}

static void tune_cache_store(const std::string& path, const std::string& key,
                             const int cv[kSizeClasses]) {
  if (path.empty()) return;
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%s %d,%d,%d,%d\n", key.c_str(), cv[0], cv[1], cv[2], cv[3]);
  std::fclose(f);
}

// Useful flops of each size class over the given plans.
static std::vector<double> class_work(const std::vector<const HostPlan*>& parts) {
  std::vector<double> w(kSizeClasses, 0.0);
  for (const HostPlan* p : parts)
    for (const CBlock& c : p->cblocks) w[size_class(c.m, c.n)] += 2.0 * c.m * c.n * c.sk;
  return w;
}

static bsm_status time_body(const std::function<bsm_status(hipStream_t)>& body, hipStream_t s,
                            int reps, float* ms) {
  hipEvent_t e0, e1;
  BSM_HIP(hipEventCreate(&e0), "hipEventCreate");
  BSM_HIP(hipEventCreate(&e1), "hipEventCreate");
  bsm_status st = body(s);  // warm-up
  if (st == BSM_OK) {
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && st == BSM_OK; ++r) st = body(s);
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    (void)hipEventElapsedTime(ms, e0, e1);
    *ms /= float(reps);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

// Timed repetitions per tile variant (after one warm-up run).
constexpr int kTuneReps = 5;

static int num_variants(int precision) {
  return precision == BSM_BF16X3 ? kNumBf16Variants : kNumVariants;
}

// Per-size-class tuning by coordinate descent: the classes that carry work, most work first, each
// try every variant with the other classes fixed (recut re-cuts and re-uploads the tasks for a
// choice of class variants, timeit times the whole product); cv holds the start and the result.
static bsm_status tune_classes(int nvar, const std::vector<double>& work, int cv[kSizeClasses],
                               const std::function<bsm_status(const int*)>& recut,
                               const std::function<bsm_status(float*)>& timeit) {
  std::vector<int> order;
  for (int c = 0; c < kSizeClasses; ++c)
    if (work[size_t(c)] > 0) order.push_back(c);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[size_t(a)] > work[size_t(b)]; });
  bsm_status st;
  for (int c : order) {
    int best = cv[c];
    float best_ms = 0.f;
    for (int v = 0; v < nvar; ++v) {
      cv[c] = v;
      if ((st = recut(cv)) != BSM_OK) return st;
      float ms = 0.f;
      if ((st = timeit(&ms)) != BSM_OK) return st;
      if (v == 0 || ms < best_ms) {
        best_ms = ms;
        best = v;
      }
    }
    cv[c] = best;
  }
  return recut(cv);
}

static int32_t reported_tile(const HostPlan& h) {
  const int v = h.uniform_variant();
  return v < 0 ? 0 : v + 1;
}

// ------------------------------------------------------------------------------------------------
// Task cost model (S10): network parameters and Adam state on the device, the feature/target
// normalisation on the host.
struct bsm_costmodel {
  std::vector<float> params;      // host copy, kept in sync with d_params
  MlpNorm norm{};
  float* d_params = nullptr;
  float* d_m = nullptr;
  float* d_v = nullptr;
  float* d_grad = nullptr;
  int64_t step = 0;               // Adam updates so far
};

static MlpNorm identity_norm() {
  MlpNorm n{};
  for (int f = 0; f < kMlpIn; ++f) {
    n.fmean[f] = 0.f;
    n.fstd[f] = 1.f;
  }
  n.tmean = 0.f;
  n.tstd = 1.f;
  return n;
}

// splitmix64: the counter-based generator behind the initial weights
static uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

static bsm_status model_device(bsm_costmodel* m) {
  if (m->d_params) return BSM_OK;
  int dev;
  bsm_status st = check_device(&dev);
  if (st != BSM_OK) return st;
  const size_t bytes = size_t(kMlpParams) * 4;
  BSM_HIP(hipMalloc(&m->d_params, bytes), "hipMalloc(model)");
  BSM_HIP(hipMalloc(&m->d_m, bytes), "hipMalloc(model)");
  BSM_HIP(hipMalloc(&m->d_v, bytes), "hipMalloc(model)");
  BSM_HIP(hipMalloc(&m->d_grad, bytes), "hipMalloc(model)");
  BSM_HIP(hipMemcpy(m->d_params, m->params.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy(model)");
  std::vector<float> z(size_t(kMlpParams), 0.f);
  BSM_HIP(hipMemcpy(m->d_m, z.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy(model)");
  BSM_HIP(hipMemcpy(m->d_v, z.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy(model)");
  return BSM_OK;
}

// Predicted log run time of n tasks (features host, n x 5) on the device; out host (n floats).
static bsm_status model_predict(bsm_costmodel* m, const float* features, int64_t n, float* out,
                                hipStream_t s) {
  if (n == 0) return BSM_OK;
  bsm_status st = model_device(m);
  if (st != BSM_OK) return st;
  float *dx = nullptr, *dy = nullptr;
  BSM_HIP(hipMalloc(&dx, size_t(n) * kMlpIn * 4), "hipMalloc(features)");
  hipError_t e = hipMalloc(&dy, size_t(n) * 4);
  if (e == hipSuccess) e = hipMemcpyAsync(dx, features, size_t(n) * kMlpIn * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_mlp_forward(m->d_params, dx, n, dy, m->norm, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out, dy, size_t(n) * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(dx);
  if (dy) (void)hipFree(dy);
  if (e != hipSuccess) return hip_fail(e, "cost model inference");
  return BSM_OK;
}

static bsm_status apply_model(HostPlan& h, bsm_costmodel* m, hipStream_t s) {
  const int64_t n = int64_t(h.items.size());
  std::vector<float> pred(static_cast<size_t>(n));
  bsm_status st = model_predict(m, h.features.data(), n, pred.data(), s);
  if (st != BSM_OK) return st;
  std::vector<double> c(pred.size());
  for (size_t q = 0; q < pred.size(); ++q) c[q] = std::exp(double(std::min(pred[q], 80.f)));
  schedule(h, c);
  return BSM_OK;
}

// ------------------------------------------------------------------------------------------------
// Allocation-free execution.  bsm_execute_static places everything the plan would otherwise
// allocate on the device -- the task list, the k-list triples, the split pass's block tables, the
// converted operands of the FP32 / split-bf16 forms and the FP64 partial sums between k-windows --
// in this one file-scope array, so that the call makes no allocation.  Each device holds its own
// copy for the life of the process.  In host code `scratch` only names the symbol: its device
// address comes from hipGetSymbolAddress, taken once per device (with that device current) and
// kept in g_scratch.
constexpr int64_t kStaticScratchBytes = int64_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch[kMaxDevices] = {};

static bsm_status scratch_of(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(BSM_E_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    BSM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch[dev]);
  return BSM_OK;
}

// Byte offsets of each buffer inside the static scratch (256-byte aligned); total = bytes used.
struct StaticLayout {
  int64_t items = 0, tri = 0, split_a = 0, split_b = 0, xpose_a = 0, xpose_b = 0, opA = 0, opB = 0,
          partial = 0, total = 0;
};

static StaticLayout static_layout(const HostPlan& h) {
  StaticLayout L;
  int64_t pos = 0;
  auto take = [&](int64_t bytes) {
    const int64_t at = pos;
    pos += (bytes + 255) / 256 * 256;
    return at;
  };
  L.items = take(int64_t(h.items.size() * sizeof(Item)));
  L.tri = take(int64_t(h.tri.size() * sizeof(Triple)));
  L.split_a = take(int64_t(h.split_a.size() * sizeof(SplitBlock)));
  L.split_b = take(int64_t(h.split_b.size() * sizeof(SplitBlock)));
  L.xpose_a = take(int64_t(h.xpose_a.size() * sizeof(XposeBlock)));
  L.xpose_b = take(int64_t(h.xpose_b.size() * sizeof(XposeBlock)));
  L.opA = take(staged_bytes(h, false));
  L.opB = take(staged_bytes(h, true));
  if (h.windows > 1) L.partial = take(h.c_elems * 8);
  L.total = pos;
  return L;
}

extern "C" {

const char* bsm_last_error(void) { return g_error.c_str(); }

bsm_status bsm_execute_static(const bsm_plan* plan, double alpha, const double* dA,
                              const double* dB, void* dC, int accumulate, void* stream) {
  if (!plan) return fail(BSM_E_INVALID, "plan is null");
  const HostPlan& h = plan->hp;
  bsm_status st = check_operands(h, dA, dB, dC, accumulate);
  if (st != BSM_OK) return st;
  if (h.dev_klists)
    return fail(BSM_E_UNSUPPORTED, "bsm_execute_static needs the k-lists in the plan's host list");
  if (h.cplx) return fail(BSM_E_UNSUPPORTED, "bsm_execute_static runs real plans only");
  if (h.ksplit > 1) return fail(BSM_E_UNSUPPORTED, "bsm_execute_static runs plans without k_split");
  const StaticLayout L = static_layout(h);
  if (L.total > kStaticScratchBytes)
    return fail(BSM_E_NOMEM, "the plan needs " + std::to_string(L.total) +
                                 " bytes of device scratch; bsm_execute_static has " +
                                 std::to_string(kStaticScratchBytes));
  if (h.items.empty()) return BSM_OK;
  int dev;
  if ((st = check_device(&dev)) != BSM_OK) return st;
  unsigned char* base = nullptr;
  if ((st = scratch_of(dev, &base)) != BSM_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // tables into the scratch (queued behind any earlier call on this stream)
  Item* items = reinterpret_cast<Item*>(base + L.items);
  Triple* tri = reinterpret_cast<Triple*>(base + L.tri);
  BSM_HIP(hipMemcpyAsync(items, h.items.data(), h.items.size() * sizeof(Item), hipMemcpyHostToDevice, s),
          "hipMemcpyAsync(tasks)");
  if (!h.tri.empty())
    BSM_HIP(hipMemcpyAsync(tri, h.tri.data(), h.tri.size() * sizeof(Triple), hipMemcpyHostToDevice, s),
            "hipMemcpyAsync(triples)");
  auto table = [&](int64_t at, const auto& v) -> bsm_status {
    if (!v.empty())
      BSM_HIP(hipMemcpyAsync(base + at, v.data(), v.size() * sizeof(v[0]), hipMemcpyHostToDevice, s),
              "hipMemcpyAsync(staging table)");
    return BSM_OK;
  };
  if ((st = table(L.split_a, h.split_a)) != BSM_OK) return st;
  if ((st = table(L.split_b, h.split_b)) != BSM_OK) return st;
  if ((st = table(L.xpose_a, h.xpose_a)) != BSM_OK) return st;
  if ((st = table(L.xpose_b, h.xpose_b)) != BSM_OK) return st;
  const Staging g{base + L.opA, base + L.opB, reinterpret_cast<const SplitBlock*>(base + L.split_a),
                  reinterpret_cast<const SplitBlock*>(base + L.split_b),
                  reinterpret_cast<const XposeBlock*>(base + L.xpose_a),
                  reinterpret_cast<const XposeBlock*>(base + L.xpose_b)};
  ProductArgs pa{};
  if ((st = convert_into(h, dA, dB, g, s, pa)) != BSM_OK) return st;
  pa.C = dC;
  pa.c_f32 = h.cfg.out_f32;
  pa.P = h.windows > 1 ? reinterpret_cast<double*>(base + L.partial) : nullptr;
  pa.alpha = alpha;
  TaskSet ts;  // views into the scratch; no counters, no clocks
  ts.items = items;
  ts.tri = tri;
  st = enqueue_tiles(h, ts, nullptr, pa, accumulate, -1, s);
  ts.items = nullptr;  // not owned
  ts.tri = nullptr;
  return st;
}

void bsm_options_default(bsm_options* opt) {
  if (!opt) return;
  opt->precision = BSM_FP64;
  opt->sched = BSM_SCHED_FLOPS;
  opt->k_window = 0;
  opt->record_timings = 0;
  opt->tile = 0;
  opt->use_graph = 0;
  opt->out = BSM_OUT_F64;
  opt->order = BSM_ORDER_DEFAULT;
  opt->patch_rows = 0;
  opt->patch_cols = 0;
  opt->device_klists = 0;
  opt->trans_a = 0;
  opt->trans_b = 0;
  opt->elem = BSM_REAL;
  opt->k_split = 0;
  opt->tune_cache = nullptr;
}

int32_t bsm_tile_variants(int32_t* tm, int32_t* tn, int32_t cap) {
  for (int v = 0; v < kNumVariants && v < cap; ++v) {
    if (tm) tm[v] = kVariants[v].tm;
    if (tn) tn[v] = kVariants[v].tn;
  }
  return kNumVariants;
}

int32_t bsm_bf16_tile_variants(int32_t* tm, int32_t* tn, int32_t cap) {
  for (int v = 0; v < kNumBf16Variants && v < cap; ++v) {
    if (tm) tm[v] = kBf16Variants[v].tm;
    if (tn) tn[v] = kBf16Variants[v].tn;
  }
  return kNumBf16Variants;
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
  if (o.use_graph != 0 && o.use_graph != 1) return fail(BSM_E_INVALID, "use_graph must be 0 or 1");
  if (o.out != BSM_OUT_F64 && o.out != BSM_OUT_F32) return fail(BSM_E_INVALID, "unknown output type");
  PlanConfig cfg;
  cfg.precision = o.precision;
  cfg.sched = o.sched;
  cfg.k_window = o.k_window;
  cfg.record_timings = o.record_timings;
  cfg.tile = o.tile;
  cfg.out_f32 = o.out == BSM_OUT_F32;
  switch (o.order) {
    case BSM_ORDER_DEFAULT: cfg.order = ORDER_AUTO; break;
    case BSM_ORDER_INTERLEAVE: cfg.order = ORDER_INTERLEAVE; break;
    case BSM_ORDER_LOCALITY: cfg.order = ORDER_LOCALITY; break;
    case BSM_ORDER_LPT: cfg.order = ORDER_LPT; break;
    case BSM_ORDER_PATCH: cfg.order = ORDER_PATCH; break;
    default: return fail(BSM_E_INVALID, "unknown task order");
  }
  if (o.patch_rows < 0 || o.patch_cols < 0) return fail(BSM_E_INVALID, "patch sizes must be >= 0");
  if (o.patch_rows > 0) cfg.patch_r = o.patch_rows;
  if (o.patch_cols > 0) cfg.patch_c = o.patch_cols;
  cfg.device_klists = o.device_klists;
  if (o.elem != BSM_REAL && o.elem != BSM_COMPLEX) return fail(BSM_E_INVALID, "unknown element type");
  cfg.k_split = o.k_split;
  cfg.cplx = o.elem == BSM_COMPLEX;
  // for real elements the adjoint is the transpose
  cfg.trans_a = (!cfg.cplx && o.trans_a == 2) ? 1 : o.trans_a;
  cfg.trans_b = (!cfg.cplx && o.trans_b == 2) ? 1 : o.trans_b;
  if (o.tune_cache) cfg.tune_cache = o.tune_cache;
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
  p->use_graph = o.use_graph;
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
  info->a_elems = h.user_a();
  info->b_elems = h.user_b();
  info->c_elems = h.user_c();
  info->triples = h.triples_total;
  info->tasks = int64_t(h.items.size());
  info->useful_flops = h.useful_flops;
  int64_t ws = int64_t(h.items.size() * sizeof(Item) + h.tri.size() * sizeof(Triple));
  if (h.dev_klists)
    ws += h.tri_capacity * int64_t(sizeof(Triple)) + int64_t(h.jobs.size() * sizeof(KJob)) +
          int64_t((h.a_bits.size() + h.bt_bits.size()) * 8 + (h.a_tab.size() + h.bt_tab.size() + h.inner.size()) * 8);
  ws += staged_bytes(h, false) + staged_bytes(h, true) + staging_table_bytes(h) + complex_bytes(h);
  if (h.ksplit > 1) ws += h.c_elems * 8 * h.ksplit + int64_t(sizeof(ProductArgs)) * h.ksplit;
  if (h.windows > 1) ws += h.c_elems * 8;
  if (h.cfg.record_timings) ws += int64_t(h.items.size()) * 16;
  info->workspace_bytes = ws;
  info->k_windows = h.windows;
  info->tile = reported_tile(h);
  info->out = h.user_out_f32() ? BSM_OUT_F32 : BSM_OUT_F64;
  info->device_klists = h.dev_klists ? 1 : 0;
  info->elem = h.cplx ? BSM_COMPLEX : BSM_REAL;
  info->k_split = h.ksplit;
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
  if (plan->hp.cplx)  // the real product's [Re; Im] block sits at twice the complex offset
    for (size_t q = 0; q < plan->hp.c_off.size(); ++q)
      if (c_offsets[q] >= 0) c_offsets[q] /= 2;
  return BSM_OK;
}

static bsm_status enqueue_product(bsm_plan* plan, double ar, double ai, const double* dA,
                                  const double* dB, void* dC, int accumulate, int skip,
                                  hipStream_t q) {
  const HostPlan& h = plan->hp;
  const double* xA = dA;
  const double* xB = dB;
  if (h.cplx) {
    BSM_HIP(launch_embed_complex(plan->d_zembed_a, int64_t(h.zembed_a.size()), dA, plan->d_zA, q),
            "embed A");
    BSM_HIP(launch_embed_complex(plan->d_zembed_b, int64_t(h.zembed_b.size()), dB, plan->d_zB, q),
            "embed B");
    xA = plan->d_zA;
    xB = plan->d_zB;
  }
  ProductArgs pa{};
  bsm_status r = enqueue_convert(plan, xA, xB, q, pa);
  if (r != BSM_OK) return r;
  pa.C = h.cplx ? static_cast<void*>(plan->d_zP) : dC;
  pa.c_f32 = h.cfg.out_f32;
  pa.P = plan->d_partial;
  pa.alpha = h.cplx ? 1.0 : ar;
  if (h.ksplit > 1) {
    // pieces into their partial buffers (absent pieces leave zeros), then their ordered sum
    BSM_HIP(launch_fill_zero(plan->d_splitP, h.c_elems * h.ksplit, q), "clear partial sums");
    r = enqueue_tiles(h, plan->ts, plan->d_kprods, pa, 0, skip, q, &plan->dk);
    if (r != BSM_OK) return r;
    plan->kprods_used = true;
    BSM_HIP(launch_reduce_splits(plan->d_splitP, h.ksplit, h.c_elems, pa.C, pa.c_f32, pa.alpha,
                                 h.cplx ? 0 : accumulate, q), "sum partial sums");
  } else {
    r = enqueue_tiles(h, plan->ts, nullptr, pa, h.cplx ? 0 : accumulate, skip, q, &plan->dk);
  }
  if (r != BSM_OK || !h.cplx) return r;
  BSM_HIP(launch_complex_epilogue(plan->d_zc, int64_t(h.zc.size()), plan->d_zP, dC, h.z_out_f32,
                                  ar, ai, accumulate, q), "complex epilogue");
  return BSM_OK;
}

// Reduction variant: the operand table of the ksplit pieces (the operands as the tile kernels read
// them, piece s writing its raw sums to partial buffer s), refreshed before anything is queued
// when the operands changed; a launch still queued may read the old table, so it is waited for.
static bsm_status kprods_refresh(bsm_plan* plan, const double* dA, const double* dB,
                                 hipStream_t s) {
  const HostPlan& h = plan->hp;
  if (h.ksplit <= 1) return BSM_OK;
  ProductArgs pa{};
  bind_operands(h, h.cplx ? plan->d_zA : dA, h.cplx ? plan->d_zB : dB, staging_of(plan), pa);
  std::vector<ProductArgs> t(size_t(h.ksplit));
  for (int q = 0; q < h.ksplit; ++q) {
    t[size_t(q)] = pa;
    t[size_t(q)].C = plan->d_splitP + int64_t(q) * h.c_elems;
    t[size_t(q)].c_f32 = 0;
    t[size_t(q)].P = nullptr;
    t[size_t(q)].alpha = 1.0;
  }
  if (t.size() == plan->h_kprods.size() &&
      std::memcmp(t.data(), plan->h_kprods.data(), t.size() * sizeof(ProductArgs)) == 0)
    return BSM_OK;
  if (plan->kprods_used) BSM_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
  BSM_HIP(hipMemcpy(plan->d_kprods, t.data(), t.size() * sizeof(ProductArgs), hipMemcpyHostToDevice),
          "hipMemcpy(piece table)");
  plan->h_kprods = t;
  return BSM_OK;
}

bsm_status bsm_execute_complex(bsm_plan* plan, double alpha_re, double alpha_im, const double* dA,
                               const double* dB, void* dC, int accumulate, void* stream) {
  if (!plan) return fail(BSM_E_INVALID, "plan is null");
  const HostPlan& h = plan->hp;
  if (!h.cplx && alpha_im != 0.0)
    return fail(BSM_E_MISMATCH, "a real plan takes a real alpha");
  hipStream_t s = static_cast<hipStream_t>(stream);
  bsm_status st = check_operands(h, dA, dB, dC, accumulate);
  if (st != BSM_OK) return st;
  if ((st = prepare(plan)) != BSM_OK) return st;
  if ((st = sync_tasks(plan, s)) != BSM_OK) return st;
  if (h.items.empty()) return BSM_OK;
  if ((st = kprods_refresh(plan, dA, dB, s)) != BSM_OK) return st;
  auto body = [&](hipStream_t q) -> bsm_status {
    return enqueue_product(plan, alpha_re, alpha_im, dA, dB, dC, accumulate, plan->skip_task, q);
  };
  if (!plan->use_graph) {
    st = body(s);
  } else {
    std::vector<uint64_t> key{uint64_t(uintptr_t(dA)), uint64_t(uintptr_t(dB)), uint64_t(uintptr_t(dC)),
                              bits_of(alpha_re), bits_of(alpha_im), uint64_t(accumulate)};
    st = plan->gc.run(key, body, s);
    if (st == BSM_OK && plan->ts.stamps) plan->ts.timed = true;
  }
  if (st == BSM_OK) {
    plan->ts.used = true;
    plan->ts.expected += h.windows;
  }
  return st;
}

bsm_status bsm_execute(bsm_plan* plan, double alpha, const double* dA, const double* dB,
                       void* dC, int accumulate, void* stream) {
  return bsm_execute_complex(plan, alpha, 0.0, dA, dB, dC, accumulate, stream);
}

bsm_status bsm_plan_verify(bsm_plan* plan, void* stream) {
  if (!plan) return fail(BSM_E_INVALID, "plan is null");
  return plan->ts.verify(static_cast<hipStream_t>(stream));
}

bsm_status bsm_plan_debug_skip_task(bsm_plan* plan, int64_t task) {
  if (!plan) return fail(BSM_E_INVALID, "plan is null");
  if (task < -1 || task >= int64_t(plan->hp.items.size()))
    return fail(BSM_E_INVALID, "task must be -1 or a task index");
  plan->skip_task = int(task);
  plan->gc.invalidate();
  return BSM_OK;
}

bsm_status bsm_plan_timings(bsm_plan* plan, float* features, float* seconds, int64_t n,
                            void* stream) {
  if (!plan) return fail(BSM_E_INVALID, "plan is null");
  return timings_of(plan->hp, plan->ts, features, seconds, n, stream);
}

bsm_status bsm_plan_features(const bsm_plan* plan, float* features, int64_t n) {
  if (!plan) return fail(BSM_E_INVALID, "plan is null");
  if (n != int64_t(plan->hp.items.size())) return fail(BSM_E_MISMATCH, "n must equal the task count");
  if (n > 0 && !features) return fail(BSM_E_INVALID, "null output");
  if (n > 0) std::memcpy(features, plan->hp.features.data(), size_t(n) * 5 * sizeof(float));
  return BSM_OK;
}

bsm_status bsm_plan_set_costs(bsm_plan* plan, const float* costs, int64_t n) {
  if (!plan) return fail(BSM_E_INVALID, "plan is null");
  bsm_status st = set_costs(plan->hp, costs, n);
  if (st == BSM_OK) plan->tasks_dirty = true;
  return st;
}

bsm_status bsm_autotune(bsm_plan* plan, const double* dA, const double* dB, void* dC,
                        void* stream, int32_t* chosen) {
  if (!plan) return fail(BSM_E_INVALID, "plan is null");
  HostPlan& h = plan->hp;
  hipStream_t s = static_cast<hipStream_t>(stream);
  bsm_status st = check_operands(h, dA, dB, dC, 0);
  if (st != BSM_OK) return st;
  if ((st = prepare(plan)) != BSM_OK) return st;
  const int nvar = num_variants(h.cfg.precision);
  const std::string key = tune_key({&h});
  int cv[kSizeClasses];
  for (int c = 0; c < kSizeClasses; ++c) cv[c] = h.class_var[c];
  auto recut = [&](const int* v) -> bsm_status {
    cut_items(h, v);
    schedule(h, flop_costs(h));
    plan->tasks_dirty = true;
    return sync_tasks(plan, s);
  };
  if ((st = kprods_refresh(plan, dA, dB, s)) != BSM_OK) return st;
  if (!tune_cache_lookup(h.cfg.tune_cache, key, nvar, cv)) {
    auto body = [&](hipStream_t q) -> bsm_status {
      return enqueue_product(plan, 1.0, 0.0, dA, dB, dC, 0, -1, q);
    };
    auto timeit = [&](float* ms) {
      plan->ts.used = true;
      return time_body(body, s, kTuneReps, ms);
    };
    if ((st = tune_classes(nvar, class_work({&h}), cv, recut, timeit)) != BSM_OK) return st;
    tune_cache_store(h.cfg.tune_cache, key, cv);
  } else if ((st = recut(cv)) != BSM_OK) {
    return st;
  }
  if (chosen) *chosen = reported_tile(h);
  return BSM_OK;
}

bsm_status bsm_plan_set_tile_classes(bsm_plan* plan, const int32_t* variants) {
  if (!plan || !variants) return fail(BSM_E_INVALID, "null argument");
  HostPlan& h = plan->hp;
  int cv[kSizeClasses];
  for (int c = 0; c < kSizeClasses; ++c) {
    if (variants[c] < 1 || variants[c] > num_variants(h.cfg.precision))
      return fail(BSM_E_INVALID, "tile variant of size class " + std::to_string(c) + " out of range");
    cv[c] = variants[c] - 1;
  }
  cut_items(h, cv);
  schedule(h, flop_costs(h));
  plan->tasks_dirty = true;
  return BSM_OK;
}

bsm_status bsm_plan_tile_classes(const bsm_plan* plan, int32_t* variants, int32_t cap) {
  if (!plan || (cap > 0 && !variants)) return fail(BSM_E_INVALID, "null argument");
  for (int c = 0; c < kSizeClasses && c < cap; ++c) variants[c] = plan->hp.class_var[c] + 1;
  return BSM_OK;
}

bsm_status bsm_plan_destroy(bsm_plan* plan) {
  if (!plan) return BSM_OK;
  bsm_status st = BSM_OK;
  if (plan->ready || plan->ts.items) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) st = hip_fail(e, "hipDeviceSynchronize");
    plan->gc.release();
    plan->ts.release();
  }
  const bsm_status sr = release_buffers(plan);
  if (st == BSM_OK) st = sr;
  delete plan;
  return st;
}

// ---- batches -------------------------------------------------------------------------------------
bsm_status bsm_batch_create(bsm_batch** out, bsm_plan* const* plans, int64_t n) {
  if (!out) return fail(BSM_E_INVALID, "out is null");
  *out = nullptr;
  if (n <= 0 || !plans) return fail(BSM_E_INVALID, "a batch needs at least one plan");
  std::vector<const HostPlan*> parts;
  for (int64_t q = 0; q < n; ++q) {
    if (!plans[q]) return fail(BSM_E_INVALID, "null plan in batch");
    if (plans[q]->hp.cplx) return fail(BSM_E_UNSUPPORTED, "batches take real plans only");
    // the FP32 and split-bf16 forms convert a member's operands into buffers the plan owns, so a
    // plan can stand for one product of the batch only
    if (plans[q]->hp.cfg.precision != BSM_FP64)
      for (int64_t r = 0; r < q; ++r)
        if (plans[r] == plans[q])
          return fail(BSM_E_INVALID, "plan " + std::to_string(q) + " repeats plan " + std::to_string(r) +
                                         " (a FP32 or split-bf16 plan can be a batch member once)");
    parts.push_back(&plans[q]->hp);
  }
  bsm_batch* b = new (std::nothrow) bsm_batch;
  if (!b) return fail(BSM_E_NOMEM, "host allocation failed");
  int code = BSM_OK;
  std::string err;
  try {
    err = merge_plans(b->hp, parts, &code);
  } catch (const std::bad_alloc&) {
    code = BSM_E_NOMEM;
    err = "host allocation failed while merging";
  }
  if (code != BSM_OK) {
    delete b;
    return fail(bsm_status(code), err);
  }
  b->members.assign(plans, plans + n);
  *out = b;
  return BSM_OK;
}

bsm_status bsm_batch_query(const bsm_batch* batch, int64_t* tasks, double* useful_flops,
                           int32_t* tile) {
  if (!batch) return fail(BSM_E_INVALID, "batch is null");
  if (tasks) *tasks = int64_t(batch->hp.items.size());
  if (useful_flops) *useful_flops = batch->hp.useful_flops;
  if (tile) *tile = reported_tile(batch->hp);
  return BSM_OK;
}

static bsm_status batch_sync(bsm_batch* b, hipStream_t stream) {
  if (!b->tasks_dirty) return BSM_OK;
  bsm_status st = b->ts.upload(b->hp, b->members[0]->hp.cfg.record_timings != 0, stream);
  if (st != BSM_OK) return st;
  b->tasks_dirty = false;
  b->gc.invalidate();
  return BSM_OK;
}

static bsm_status batch_body(bsm_batch* b, const double* const* dA, const double* const* dB,
                             int accumulate, hipStream_t s) {
  for (size_t q = 0; q < b->members.size(); ++q) {
    ProductArgs pa{};
    bsm_status st = enqueue_convert(b->members[q], dA[q], dB[q], s, pa);
    if (st != BSM_OK) return st;
  }
  return enqueue_tiles(b->hp, b->ts, b->d_prods, ProductArgs{}, accumulate, -1, s);
}

// Operand table of the batch (device copy refreshed only when a pointer or alpha changed; a
// launch queued on `stream` may still read the old one, so it is waited for first).
static bsm_status batch_table(bsm_batch* b, const double* alphas, const double* const* dA,
                              const double* const* dB, void* const* dC, hipStream_t stream) {
  const size_t n = b->members.size();
  std::vector<ProductArgs> t(n);
  for (size_t q = 0; q < n; ++q) {
    bsm_plan* p = b->members[q];
    const HostPlan& h = p->hp;
    ProductArgs& pa = t[q];
    std::memset(&pa, 0, sizeof pa);
    bind_operands(h, dA[q], dB[q], staging_of(p), pa);
    pa.C = dC[q];
    pa.c_f32 = h.cfg.out_f32;
    pa.P = nullptr;
    pa.alpha = alphas ? alphas[q] : 1.0;
  }
  bool same = t.size() == b->h_prods.size() && b->d_prods &&
              std::memcmp(t.data(), b->h_prods.data(), n * sizeof(ProductArgs)) == 0;
  if (!same) {
    if (b->table_used) BSM_HIP(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (!b->d_prods) BSM_HIP(hipMalloc(&b->d_prods, n * sizeof(ProductArgs)), "hipMalloc(operand table)");
    BSM_HIP(hipMemcpy(b->d_prods, t.data(), n * sizeof(ProductArgs), hipMemcpyHostToDevice),
            "hipMemcpy(operand table)");
    b->h_prods = t;
  }
  return BSM_OK;
}

bsm_status bsm_batch_execute(bsm_batch* batch, const double* alphas, const double* const* dA,
                             const double* const* dB, void* const* dC, int accumulate,
                             void* stream) {
  if (!batch) return fail(BSM_E_INVALID, "batch is null");
  if (!dA || !dB || !dC) return fail(BSM_E_INVALID, "null operand array");
  hipStream_t s = static_cast<hipStream_t>(stream);
  bsm_status st;
  for (size_t q = 0; q < batch->members.size(); ++q) {
    if ((st = check_operands(batch->members[q]->hp, dA[q], dB[q], dC[q], accumulate)) != BSM_OK) return st;
    if ((st = prepare(batch->members[q])) != BSM_OK) return st;
  }
  if ((st = batch_sync(batch, s)) != BSM_OK) return st;
  if ((st = batch_table(batch, alphas, dA, dB, dC, s)) != BSM_OK) return st;
  if (batch->hp.items.empty()) return BSM_OK;
  // one graph: every member's operand conversion, then one tile launch over all tasks
  std::vector<uint64_t> key{uint64_t(accumulate)};
  for (size_t q = 0; q < batch->members.size(); ++q) {
    key.push_back(uint64_t(uintptr_t(dA[q])));
    key.push_back(uint64_t(uintptr_t(dB[q])));
    key.push_back(uint64_t(uintptr_t(dC[q])));
    key.push_back(bits_of(alphas ? alphas[q] : 1.0));
  }
  auto body = [&](hipStream_t q) { return batch_body(batch, dA, dB, accumulate, q); };
  st = batch->gc.run(key, body, s);
  if (st == BSM_OK) {
    if (batch->ts.stamps) batch->ts.timed = true;
    batch->ts.used = true;
    batch->table_used = true;
    batch->ts.expected += 1;
  }
  return st;
}

bsm_status bsm_batch_verify(bsm_batch* batch, void* stream) {
  if (!batch) return fail(BSM_E_INVALID, "batch is null");
  return batch->ts.verify(static_cast<hipStream_t>(stream));
}

bsm_status bsm_batch_timings(bsm_batch* batch, float* features, float* seconds, int64_t n,
                             void* stream) {
  if (!batch) return fail(BSM_E_INVALID, "batch is null");
  return timings_of(batch->hp, batch->ts, features, seconds, n, stream);
}

bsm_status bsm_batch_set_costs(bsm_batch* batch, const float* costs, int64_t n) {
  if (!batch) return fail(BSM_E_INVALID, "batch is null");
  bsm_status st = set_costs(batch->hp, costs, n);
  if (st == BSM_OK) batch->tasks_dirty = true;
  return st;
}

bsm_status bsm_batch_autotune(bsm_batch* batch, const double* const* dA, const double* const* dB,
                              void* const* dC, void* stream, int32_t* chosen) {
  if (!batch) return fail(BSM_E_INVALID, "batch is null");
  if (!dA || !dB || !dC) return fail(BSM_E_INVALID, "null operand array");
  hipStream_t s = static_cast<hipStream_t>(stream);
  bsm_status st;
  std::vector<const HostPlan*> parts;
  for (size_t q = 0; q < batch->members.size(); ++q) {
    if ((st = check_operands(batch->members[q]->hp, dA[q], dB[q], dC[q], 0)) != BSM_OK) return st;
    if ((st = prepare(batch->members[q])) != BSM_OK) return st;
    parts.push_back(&batch->members[q]->hp);
  }
  const int nvar = num_variants(parts[0]->cfg.precision);
  const std::string key = tune_key(parts);
  // every member is re-cut with the same class variants, then the batch is merged again
  auto recut = [&](const int* v) -> bsm_status {
    for (bsm_plan* p : batch->members) {
      cut_items(p->hp, v);
      schedule(p->hp, flop_costs(p->hp));
      p->tasks_dirty = true;
    }
    int code = BSM_OK;
    std::string err = merge_plans(batch->hp, parts, &code);
    if (code != BSM_OK) return fail(bsm_status(code), err);
    batch->tasks_dirty = true;
    return batch_sync(batch, s);
  };
  int cv[kSizeClasses];
  for (int c = 0; c < kSizeClasses; ++c) cv[c] = parts[0]->class_var[c];
  const std::string& cache = parts[0]->cfg.tune_cache;
  if (!tune_cache_lookup(cache, key, nvar, cv)) {
    if ((st = batch_table(batch, nullptr, dA, dB, dC, s)) != BSM_OK) return st;
    batch->table_used = true;
    auto body = [&](hipStream_t q) { return batch_body(batch, dA, dB, 0, q); };
    auto timeit = [&](float* ms) {
      batch->ts.used = true;
      return time_body(body, s, kTuneReps, ms);
    };
    if ((st = tune_classes(nvar, class_work(parts), cv, recut, timeit)) != BSM_OK) return st;
    tune_cache_store(cache, key, cv);
  } else if ((st = recut(cv)) != BSM_OK) {
    return st;
  }
  if (chosen) *chosen = reported_tile(batch->hp);
  return BSM_OK;
}

bsm_status bsm_batch_tile_classes(const bsm_batch* batch, int32_t* variants, int32_t cap) {
  if (!batch || (cap > 0 && !variants)) return fail(BSM_E_INVALID, "null argument");
  for (int c = 0; c < kSizeClasses && c < cap; ++c) variants[c] = batch->hp.class_var[c] + 1;
  return BSM_OK;
}

bsm_status bsm_batch_destroy(bsm_batch* batch) {
  if (!batch) return BSM_OK;
  bsm_status st = BSM_OK;
  if (batch->ts.items || batch->d_prods) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) st = hip_fail(e, "hipDeviceSynchronize");
  }
  batch->gc.release();
  batch->ts.release();
  if (batch->d_prods) (void)hipFree(batch->d_prods);
  delete batch;
  return st;
}

// ---- cost model ---------------------------------------------------------------------------------
bsm_status bsm_costmodel_create(bsm_costmodel** out, uint64_t seed) {
  if (!out) return fail(BSM_E_INVALID, "out is null");
  bsm_costmodel* m = new (std::nothrow) bsm_costmodel;
  if (!m) return fail(BSM_E_NOMEM, "host allocation failed");
  // He-uniform weights from splitmix64(seed, index); biases 0
  m->params.assign(size_t(kMlpParams), 0.f);
  const int H = kMlpHidden, F = kMlpIn;
  auto u01 = [&](uint64_t i) { return float(double(splitmix64(seed * 0x100000001B3ull + i) >> 11) * 0x1.0p-53); };
  for (int q = 0; q < H * F; ++q) m->params[size_t(q)] = (2.f * u01(uint64_t(q)) - 1.f) * std::sqrt(6.f / F);
  const int ow2 = H * F + H;
  for (int q = 0; q < H * H; ++q) m->params[size_t(ow2 + q)] = (2.f * u01(uint64_t(ow2 + q)) - 1.f) * std::sqrt(6.f / H);
  const int ow3 = ow2 + H * H + H;
  for (int q = 0; q < H; ++q) m->params[size_t(ow3 + q)] = (2.f * u01(uint64_t(ow3 + q)) - 1.f) * std::sqrt(6.f / H);
  m->norm = identity_norm();
  *out = m;
  return BSM_OK;
}

int64_t bsm_costmodel_param_count(void) { return kMlpParams; }

bsm_status bsm_costmodel_params(const bsm_costmodel* m, float* params, int64_t n, float* norm12) {
  if (!m) return fail(BSM_E_INVALID, "model is null");
  if (params) {
    if (n != kMlpParams) return fail(BSM_E_MISMATCH, "n must equal bsm_costmodel_param_count()");
    std::memcpy(params, m->params.data(), size_t(kMlpParams) * 4);
  }
  if (norm12) {
    for (int f = 0; f < kMlpIn; ++f) {
      norm12[f] = m->norm.fmean[f];
      norm12[kMlpIn + f] = m->norm.fstd[f];
    }
    norm12[2 * kMlpIn] = m->norm.tmean;
    norm12[2 * kMlpIn + 1] = m->norm.tstd;
  }
  return BSM_OK;
}

bsm_status bsm_costmodel_set_params(bsm_costmodel* m, const float* params, int64_t n,
                                    const float* norm12) {
  if (!m) return fail(BSM_E_INVALID, "model is null");
  if (params) {
    if (n != kMlpParams) return fail(BSM_E_MISMATCH, "n must equal bsm_costmodel_param_count()");
    m->params.assign(params, params + kMlpParams);
    if (m->d_params)
      BSM_HIP(hipMemcpy(m->d_params, params, size_t(kMlpParams) * 4, hipMemcpyHostToDevice), "hipMemcpy(model)");
  }
  if (norm12) {
    for (int f = 0; f < kMlpIn; ++f) {
      if (!(norm12[kMlpIn + f] > 0.f)) return fail(BSM_E_INVALID, "feature scales must be > 0");
      m->norm.fmean[f] = norm12[f];
      m->norm.fstd[f] = norm12[kMlpIn + f];
    }
    if (!(norm12[2 * kMlpIn + 1] > 0.f)) return fail(BSM_E_INVALID, "target scale must be > 0");
    m->norm.tmean = norm12[2 * kMlpIn];
    m->norm.tstd = norm12[2 * kMlpIn + 1];
  }
  return BSM_OK;
}

bsm_status bsm_costmodel_train(bsm_costmodel* m, const float* features, const float* log_seconds,
                               int64_t n, int64_t epochs, int64_t batch, float lr,
                               float* final_loss, void* stream) {
  if (!m) return fail(BSM_E_INVALID, "model is null");
  if (n <= 0 || !features || !log_seconds) return fail(BSM_E_INVALID, "empty training set");
  if (epochs < 0 || batch <= 0 || !(lr > 0.f)) return fail(BSM_E_INVALID, "epochs >= 0, batch > 0, lr > 0");
  bsm_status st = model_device(m);
  if (st != BSM_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // normalisation statistics of this training set (means and standard deviations)
  MlpNorm nm{};
  for (int f = 0; f < kMlpIn; ++f) {
    double mu = 0, sq = 0;
    for (int64_t q = 0; q < n; ++q) mu += features[q * kMlpIn + f];
    mu /= double(n);
    for (int64_t q = 0; q < n; ++q) sq += (features[q * kMlpIn + f] - mu) * (features[q * kMlpIn + f] - mu);
    double sd = std::sqrt(sq / double(n));
    nm.fmean[f] = float(mu);
    nm.fstd[f] = float(sd > 1e-6 ? sd : 1.0);
  }
  {
    double mu = 0, sq = 0;
    for (int64_t q = 0; q < n; ++q) mu += log_seconds[q];
    mu /= double(n);
    for (int64_t q = 0; q < n; ++q) sq += (log_seconds[q] - mu) * (log_seconds[q] - mu);
    double sd = std::sqrt(sq / double(n));
    nm.tmean = float(mu);
    nm.tstd = float(sd > 1e-6 ? sd : 1.0);
  }
  m->norm = nm;
  const int64_t bmax = std::min(batch, n);
  float *dx = nullptr, *dt = nullptr, *part = nullptr, *pl = nullptr, *dloss = nullptr;
  hipError_t e = hipMalloc(&dx, size_t(n) * kMlpIn * 4);
  if (e == hipSuccess) e = hipMalloc(&dt, size_t(n) * 4);
  const int64_t rows = mlp_partial_rows(std::max(bmax, n));
  if (e == hipSuccess) e = hipMalloc(&part, size_t(rows) * kMlpParams * 4);
  if (e == hipSuccess) e = hipMalloc(&pl, size_t(rows) * 4);
  if (e == hipSuccess) e = hipMalloc(&dloss, 4);
  if (e == hipSuccess) e = hipMemcpyAsync(dx, features, size_t(n) * kMlpIn * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dt, log_seconds, size_t(n) * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_mlp_normalize(dx, dt, n, nm, s);
  // mini-batches in a fixed order; Adam after each
  for (int64_t ep = 0; ep < epochs && e == hipSuccess; ++ep)
    for (int64_t b0 = 0; b0 < n && e == hipSuccess; b0 += bmax) {
      const int64_t cnt = std::min(bmax, n - b0);
      e = launch_mlp_loss_grad(m->d_params, dx + b0 * kMlpIn, dt + b0, cnt, part, pl, m->d_grad,
                               nullptr, s);
      if (e == hipSuccess)
        e = launch_adam(m->d_params, m->d_grad, m->d_m, m->d_v, kMlpParams, ++m->step, lr, 0.9f,
                        0.999f, 1e-8f, s);
    }
  float loss = 0.f;
  if (e == hipSuccess) e = launch_mlp_loss_grad(m->d_params, dx, dt, n, part, pl, m->d_grad, dloss, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&loss, dloss, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(m->params.data(), m->d_params, size_t(kMlpParams) * 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  for (float* ptr : {dx, dt, part, pl, dloss})
    if (ptr) (void)hipFree(ptr);
  if (e != hipSuccess) return hip_fail(e, "cost model training");
  if (final_loss) *final_loss = loss;  // mean squared error in normalised log-time units
  return BSM_OK;
}

bsm_status bsm_costmodel_predict(bsm_costmodel* m, const float* features, int64_t n,
                                 float* log_seconds, void* stream) {
  if (!m) return fail(BSM_E_INVALID, "model is null");
  if (n < 0 || (n > 0 && (!features || !log_seconds))) return fail(BSM_E_INVALID, "null argument");
  return model_predict(m, features, n, log_seconds, static_cast<hipStream_t>(stream));
}

bsm_status bsm_costmodel_save(const bsm_costmodel* m, const char* path) {
  if (!m || !path) return fail(BSM_E_INVALID, "null argument");
  std::vector<float> mv(size_t(2 * kMlpParams), 0.f);
  if (m->d_m) {
    BSM_HIP(hipMemcpy(mv.data(), m->d_m, size_t(kMlpParams) * 4, hipMemcpyDeviceToHost), "hipMemcpy(model)");
    BSM_HIP(hipMemcpy(mv.data() + kMlpParams, m->d_v, size_t(kMlpParams) * 4, hipMemcpyDeviceToHost), "hipMemcpy(model)");
  }
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(BSM_E_INVALID, std::string("cannot open ") + path);
  const char magic[8] = {'B', 'S', 'M', 'C', 'M', '0', '0', '1'};
  const int32_t count = kMlpParams;
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(&count, 4, 1, f) == 1 &&
            std::fwrite(&m->step, 8, 1, f) == 1 && std::fwrite(&m->norm, sizeof(MlpNorm), 1, f) == 1 &&
            std::fwrite(m->params.data(), 4, size_t(kMlpParams), f) == size_t(kMlpParams) &&
            std::fwrite(mv.data(), 4, mv.size(), f) == mv.size();
  ok = (std::fclose(f) == 0) && ok;
  return ok ? BSM_OK : fail(BSM_E_INVALID, std::string("write failed: ") + path);
}

bsm_status bsm_costmodel_load(bsm_costmodel** out, const char* path) {
  if (!out || !path) return fail(BSM_E_INVALID, "null argument");
  *out = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(BSM_E_INVALID, std::string("cannot open ") + path);
  char magic[8];
  int32_t count = 0;
  bsm_costmodel* m = new (std::nothrow) bsm_costmodel;
  if (!m) {
    std::fclose(f);
    return fail(BSM_E_NOMEM, "host allocation failed");
  }
  m->params.assign(size_t(kMlpParams), 0.f);
  std::vector<float> mv(size_t(2 * kMlpParams));
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "BSMCM001", 8) == 0 &&
            std::fread(&count, 4, 1, f) == 1 && count == kMlpParams &&
            std::fread(&m->step, 8, 1, f) == 1 && std::fread(&m->norm, sizeof(MlpNorm), 1, f) == 1 &&
            std::fread(m->params.data(), 4, size_t(kMlpParams), f) == size_t(kMlpParams) &&
            std::fread(mv.data(), 4, mv.size(), f) == mv.size();
  std::fclose(f);
  if (!ok) {
    delete m;
    return fail(BSM_E_INVALID, std::string("not a cost model file: ") + path);
  }
  bsm_status st = model_device(m);
  if (st == BSM_OK) {
    hipError_t e = hipMemcpy(m->d_m, mv.data(), size_t(kMlpParams) * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->d_v, mv.data() + kMlpParams, size_t(kMlpParams) * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) st = hip_fail(e, "hipMemcpy(model)");
  }
  if (st != BSM_OK) {
    bsm_costmodel_destroy(m);
    return st;
  }
  *out = m;
  return BSM_OK;
}

bsm_status bsm_costmodel_destroy(bsm_costmodel* m) {
  if (!m) return BSM_OK;
  for (float* ptr : {m->d_params, m->d_m, m->d_v, m->d_grad})
    if (ptr) (void)hipFree(ptr);
  delete m;
  return BSM_OK;
}

bsm_status bsm_plan_set_costmodel(bsm_plan* plan, bsm_costmodel* model, void* stream) {
  if (!plan || !model) return fail(BSM_E_INVALID, "null argument");
  bsm_status st = apply_model(plan->hp, model, static_cast<hipStream_t>(stream));
  if (st == BSM_OK) {
    plan->tasks_dirty = true;
    plan->hp.cfg.sched = BSM_SCHED_MLP;
  }
  return st;
}

bsm_status bsm_batch_set_costmodel(bsm_batch* batch, bsm_costmodel* model, void* stream) {
  if (!batch || !model) return fail(BSM_E_INVALID, "null argument");
  bsm_status st = apply_model(batch->hp, model, static_cast<hipStream_t>(stream));
  if (st == BSM_OK) {
    batch->tasks_dirty = true;
    batch->hp.cfg.sched = BSM_SCHED_MLP;
  }
  return st;
}

// Device-pointer entry points of the network itself (no normalisation), for checking its
// arithmetic: forward, mean-squared-error loss with gradient, and one Adam step.
bsm_status bsm_mlp_forward(const float* d_params, const float* d_x, int64_t n, float* d_y,
                           void* stream) {
  if (n < 0 || (n > 0 && (!d_params || !d_x || !d_y))) return fail(BSM_E_INVALID, "null argument");
  int dev;
  bsm_status st = check_device(&dev);
  if (st != BSM_OK) return st;
  BSM_HIP(launch_mlp_forward(d_params, d_x, n, d_y, identity_norm(), static_cast<hipStream_t>(stream)),
          "mlp forward");
  return BSM_OK;
}

bsm_status bsm_mlp_loss_grad(const float* d_params, const float* d_x, const float* d_t, int64_t n,
                             float* d_grad, float* d_loss, void* stream) {
  if (n <= 0 || !d_params || !d_x || !d_t || !d_grad) return fail(BSM_E_INVALID, "null argument");
  int dev;
  bsm_status st = check_device(&dev);
  if (st != BSM_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t rows = mlp_partial_rows(n);
  float *part = nullptr, *pl = nullptr;
  hipError_t e = hipMalloc(&part, size_t(rows) * kMlpParams * 4);
  if (e == hipSuccess) e = hipMalloc(&pl, size_t(rows) * 4);
  if (e == hipSuccess) e = launch_mlp_loss_grad(d_params, d_x, d_t, n, part, pl, d_grad, d_loss, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the workspace is freed below
  if (part) (void)hipFree(part);
  if (pl) (void)hipFree(pl);
  if (e != hipSuccess) return hip_fail(e, "mlp loss/gradient");
  return BSM_OK;
}

bsm_status bsm_adam_step(float* d_params, const float* d_grad, float* d_m, float* d_v, int64_t n,
                         int64_t step, float lr, float beta1, float beta2, float eps, void* stream) {
  if (n < 0 || step < 1 || (n > 0 && (!d_params || !d_grad || !d_m || !d_v)))
    return fail(BSM_E_INVALID, "bad argument");
  int dev;
  bsm_status st = check_device(&dev);
  if (st != BSM_OK) return st;
  BSM_HIP(launch_adam(d_params, d_grad, d_m, d_v, n, step, lr, beta1, beta2, eps,
                      static_cast<hipStream_t>(stream)),
          "adam");
  return BSM_OK;
}

}  // extern "C"
