// Host planner.  Paper Sec. 3.2: the matrices are over-decomposed into problem-given blocks and
// each rank-k update is split into per-block multiply tasks; Fig. 3 splits one iteration into
// tasks that each produce one piece of the process's part of C.  Here a task is a sub-tile of
// one present C block together with that block's whole k-list, so the multiply and the reduction
// into C are one task (no temporaries, one writer per C element).
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <thread>
#include <tuple>

#include "../../include/bsm.h"
#include "staging.hpp"

namespace bsm {

int64_t words_for(int64_t ncols) { return (ncols + 63) / 64; }

static inline bool test_bit(const uint64_t* bits, int64_t wpr, int64_t i, int64_t j) {
  return (bits[i * wpr + (j >> 6)] >> (j & 63)) & 1u;
}

static std::string check_tiling(const char* name, int64_t n, const int64_t* sz) {
  if (n < 0) return std::string(name) + ": negative block count";
  if (n > 0 && !sz) return std::string(name) + ": null size vector";
  for (int64_t i = 0; i < n; ++i)
    if (sz[i] < 1 || sz[i] > kMaxBlock)
      return std::string(name) + ": block " + std::to_string(i) + " has size " +
             std::to_string(sz[i]) + " (allowed 1.." + std::to_string(kMaxBlock) + ")";
  return "";
}

static std::string check_bits(const char* name, int64_t r, int64_t c, const uint64_t* bits) {
  int64_t w = words_for(c);
  if (r * w == 0) return "";
  if (!bits) return std::string(name) + ": null bitmap";
  if (c % 64) {
    uint64_t pad = ~uint64_t(0) << (c % 64);
    for (int64_t i = 0; i < r; ++i)
      if (bits[i * w + w - 1] & pad)
        return std::string(name) + ": padding bit set in row " + std::to_string(i);
  }
  return "";
}

// Packed offsets of the present blocks (row-major block order); returns the element count.
static int64_t pack_offsets(int64_t R, int64_t C, const std::vector<int64_t>& rsz,
                            const std::vector<int64_t>& csz, const std::vector<uint64_t>& bits,
                            std::vector<int64_t>& off, int64_t& nblocks) {
  off.assign(size_t(R * C), -1);
  int64_t w = words_for(C), pos = 0;
  nblocks = 0;
  for (int64_t i = 0; i < R; ++i)
    for (int64_t j = 0; j < C; ++j)
      if (test_bit(bits.data(), w, i, j)) {
        off[size_t(i * C + j)] = pos;
        pos += rsz[size_t(i)] * csz[size_t(j)];
        ++nblocks;
      }
  return pos;
}

// The R x C shape `bits` transposed (C x R, same word layout).
static std::vector<uint64_t> transpose_bits(const uint64_t* bits, int64_t R, int64_t C) {
  const int64_t wc = words_for(C), wr = words_for(R);
  std::vector<uint64_t> out(size_t(C * wr), 0);
  for (int64_t i = 0; i < R; ++i)
    for (int64_t w = 0; w < wc; ++w) {
      uint64_t x = bits[i * wc + w];
      while (x) {
        const int64_t j = w * 64 + __builtin_ctzll(x);
        x &= x - 1;
        out[size_t(j * wr + (i >> 6))] |= uint64_t(1) << (i & 63);
      }
    }
  return out;
}

// Sub-tile cuts of one C block: a dimension of nb16 16-row blocks is cut into the fewest pieces
// of at most `per` blocks, as equal as the 16-row granule allows (larger pieces first).
static void cut_dim(int m, int per, std::vector<std::pair<int, int>>& out) {
  out.clear();
  const int nb16 = (m + 15) / 16;
  const int parts = (nb16 + per - 1) / per;
  const int base = nb16 / parts, extra = nb16 % parts;
  int off = 0;
  for (int q = 0; q < parts; ++q) {
    const int nb = base + (q < extra ? 1 : 0);
    out.emplace_back(off, std::min(nb * 16, m - off));
    off += nb * 16;
  }
}

std::vector<double> flop_costs(const HostPlan& p) {
  std::vector<double> c(p.items.size());
  for (size_t q = 0; q < p.items.size(); ++q) c[q] = 2.0 * p.items[q].h * p.items[q].w * p.meta[q].sk;
  return c;
}

// Device-built k-lists: every segment is cut into batches whose C blocks' triples fit the
// device's triple buffer.  A batch takes C blocks (with all their tasks) from the fronts of the
// segment's XCD runs until the next one would overflow the buffer, so that every batch takes at
// least one block; it becomes a segment of its own.
// Each batch gets one job per distinct C block, and its tasks point into the job's range of the
// buffer.
static void batch_device_klists(HostPlan& p) {
  const int64_t budget = p.cfg.device_klists >= 2 ? p.cfg.device_klists : kDeviceTriples;
  std::vector<Item> items;
  std::vector<ItemMeta> metas;
  std::vector<double> costs;
  std::vector<float> feats;
  std::vector<Segment> segs;
  p.jobs.clear();
  p.tri_capacity = 0;
  items.reserve(p.items.size());
  metas.reserve(p.items.size());
  costs.reserve(p.items.size());
  feats.reserve(p.features.size());
  for (const Segment& g : p.segs) {
    int32_t pos[kXcds], end[kXcds];
    for (int x = 0; x < kXcds; ++x) {
      pos[x] = g.begin + g.xcd_begin[x];
      end[x] = g.begin + g.xcd_begin[x + 1];
    }
    // tasks [q, run_end(q)) belong to one C block
    auto run_end = [&](int32_t q, int32_t e) {
      int32_t r = q + 1;
      while (r < e && p.items[size_t(r)].c_off == p.items[size_t(q)].c_off &&
             p.items[size_t(r)].product == p.items[size_t(q)].product)
        ++r;
      return r;
    };
    for (;;) {
      bool left = false;
      for (int x = 0; x < kXcds; ++x) left = left || pos[x] < end[x];
      if (!left) break;
      // this batch's share of every run: [pos[x], stop[x])
      int32_t stop[kXcds];
      for (int x = 0; x < kXcds; ++x) stop[x] = pos[x];
      // the next C block comes from the run whose share of this batch costs least so far (the
      // scheduler's costs), so that every batch keeps the XCDs balanced
      int64_t tri = 0;
      double load[kXcds] = {0};
      for (;;) {
        int best = -1;
        for (int x = 0; x < kXcds; ++x)
          if (stop[x] < end[x] && (best < 0 || load[x] < load[best])) best = x;
        if (best < 0) break;
        const int64_t c = p.items[size_t(stop[best])].tri_count;
        if (tri > 0 && tri + c > budget) break;
        tri += c;
        const int32_t e = run_end(stop[best], end[best]);
        for (int32_t q = stop[best]; q < e; ++q) load[best] += p.cost[size_t(q)];
        stop[best] = e;
      }
      Segment b;
      b.variant = g.variant;
      b.begin = int32_t(items.size());
      b.job_begin = int64_t(p.jobs.size());
      std::map<std::pair<uint32_t, int64_t>, size_t> job_of;  // (product, C offset) -> job
      uint32_t used = 0;
      int64_t maxc = 0;
      for (int x = 0; x < kXcds; ++x) {
        b.xcd_begin[x] = int32_t(items.size()) - b.begin;
        for (int32_t q = pos[x]; q < stop[x]; ++q) {
          Item it = p.items[size_t(q)];
          const auto key = std::make_pair(it.product, it.c_off);
          auto f = job_of.find(key);
          if (f == job_of.end()) {
            f = job_of.emplace(key, p.jobs.size()).first;
            p.jobs.push_back(KJob{p.meta[size_t(q)].ci, p.meta[size_t(q)].cj, used, it.tri_count});
            used += it.tri_count;
          }
          it.tri_begin = p.jobs[f->second].tri_begin;
          items.push_back(it);
          metas.push_back(p.meta[size_t(q)]);
          costs.push_back(p.cost[size_t(q)]);
          for (int f5 = 0; f5 < 5; ++f5) feats.push_back(p.features[size_t(q) * 5 + size_t(f5)]);
        }
        maxc = std::max<int64_t>(maxc, stop[x] - pos[x]);
        pos[x] = stop[x];
      }
      b.xcd_begin[kXcds] = int32_t(items.size()) - b.begin;
      b.end = int32_t(items.size());
      b.grid = maxc * kXcds;
      b.job_count = int64_t(p.jobs.size()) - b.job_begin;
      p.tri_capacity = std::max<int64_t>(p.tri_capacity, used);
      segs.push_back(b);
    }
  }
  p.items.swap(items);
  p.meta.swap(metas);
  p.cost.swap(costs);
  p.features.swap(feats);
  p.segs.swap(segs);
}

// Deals the tasks of one segment (indices `idx` into the canonically ordered task list) to the
// XCDs; returns one list of task indices per XCD.
// Split-pass table entries of one operand block (written at plane offset dst, rows x pad_k(ks)):
// one piece per 32-wide k-panel, so that every workgroup of the pass moves at most 256 x 32
// elements whatever the block size.  A piece of a block stored rows x ks (transpose = 0) starts
// 32 columns further on; one of a block stored ks x rows (transpose = 1) 32 source rows further.
static void push_split(std::vector<SplitBlock>& out, int64_t src, int64_t dst, int64_t rows,
                       int64_t ks, int64_t ld, int transpose) {
  for (int64_t k0 = 0; k0 < ks; k0 += kSliceK)
    out.push_back(SplitBlock{src + (transpose ? k0 * ld : k0), dst + k0 * rows, int32_t(rows),
                             int32_t(std::min<int64_t>(kSliceK, ks - k0)), int32_t(ld), transpose});
}

static std::vector<std::vector<size_t>> deal(const HostPlan& p, const std::vector<size_t>& idx,
                                             const std::vector<double>& cost) {
  std::vector<std::vector<size_t>> bins(kXcds);
  std::vector<double> load(kXcds, 0.0);
  const int order = p.cfg.order != ORDER_AUTO ? p.cfg.order
                                              : (p.items.size() <= kLptTasks ? ORDER_LPT : ORDER_INTERLEAVE);
  if (order == ORDER_LPT) {
    // longest processing time first: largest task to the least-loaded XCD, each XCD then runs
    // its tasks largest first (its 32 CUs pick them up in that order)
    std::vector<size_t> o(idx);
    std::stable_sort(o.begin(), o.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
    for (size_t q : o) {
      int x = int(std::min_element(load.begin(), load.end()) - load.begin());
      bins[size_t(x)].push_back(q);
      load[size_t(x)] += cost[q];
    }
  } else if (order == ORDER_PATCH) {
    // patches of patch_r x patch_c C blocks, in row-major patch order per product; each whole
    // patch to the least-loaded XCD; inside a patch the canonical C-block order (stable sort)
    const int pr = std::max(1, p.cfg.patch_r), pc = std::max(1, p.cfg.patch_c);
    auto key = [&](size_t q) {
      return std::make_tuple(p.items[q].product, p.meta[q].ci / pr, p.meta[q].cj / pc);
    };
    std::vector<size_t> o(idx);
    std::stable_sort(o.begin(), o.end(), [&](size_t a, size_t b) { return key(a) < key(b); });
    size_t u = 0;
    while (u < o.size()) {
      size_t e = u + 1;
      double c = cost[o[u]];
      while (e < o.size() && key(o[e]) == key(o[u])) c += cost[o[e++]];
      int x = int(std::min_element(load.begin(), load.end()) - load.begin());
      for (size_t r = u; r < e; ++r) bins[size_t(x)].push_back(o[r]);
      load[size_t(x)] += c;
      u = e;
    }
  } else if (order == ORDER_INTERLEAVE) {
    // whole C blocks (consecutive tasks with the same C offset) dealt to the least-loaded XCD in
    // C-block order
    size_t u = 0;
    while (u < idx.size()) {
      size_t e = u + 1;
      double c = cost[idx[u]];
      const Item& first = p.items[idx[u]];
      while (e < idx.size() && p.items[idx[e]].c_off == first.c_off &&
             p.items[idx[e]].product == first.product)
        c += cost[idx[e++]];
      int x = int(std::min_element(load.begin(), load.end()) - load.begin());
      for (size_t r = u; r < e; ++r) bins[size_t(x)].push_back(idx[r]);
      load[size_t(x)] += c;
      u = e;
    }
  } else {
    // keep the C-block order (sub-tiles of a block and blocks of a block row stay together, so
    // they share A and B tiles in one XCD's L2) and cut it into kXcds runs of equal cost
    double total = 0;
    for (size_t q : idx) total += cost[q];
    double acc = 0;
    int x = 0;
    for (size_t q : idx) {
      while (x < kXcds - 1 && acc >= total * (x + 1) / kXcds) ++x;
      bins[size_t(x)].push_back(q);
      acc += cost[q];
    }
  }
  return bins;
}

void schedule(HostPlan& p, const std::vector<double>& cost_in) {
  size_t n = p.items.size();
  // Every order below is defined on the tasks in C-block order (product, C offset, sub-tile), so
  // the tasks are put back in that order first: a reschedule then gives the same result whatever
  // order an earlier schedule left them in.
  std::vector<double> cost(cost_in);
  {
    std::vector<size_t> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](size_t a, size_t b) {
      const Item& x = p.items[a];
      const Item& y = p.items[b];
      if (x.product != y.product) return x.product < y.product;
      if (x.c_off != y.c_off) return x.c_off < y.c_off;
      if (x.r0 != y.r0) return x.r0 < y.r0;
      return x.c0 < y.c0;
    });
    std::vector<Item> it2(n);
    std::vector<ItemMeta> v2(n);
    std::vector<double> c2(n);
    std::vector<float> f2(p.features.size());
    for (size_t q = 0; q < n; ++q) {
      it2[q] = p.items[perm[q]];
      v2[q] = p.meta[perm[q]];
      c2[q] = cost_in[perm[q]];
      for (int f = 0; f < 5; ++f) f2[q * 5 + size_t(f)] = p.features[perm[q] * 5 + size_t(f)];
    }
    p.items.swap(it2);
    p.meta.swap(v2);
    p.features.swap(f2);
    cost.swap(c2);
  }
  // one segment per tile variant in use, each dealt to the XCDs on its own
  std::vector<Item> items;
  std::vector<ItemMeta> metas;
  std::vector<double> c2;
  std::vector<float> f2;
  items.reserve(n);
  metas.reserve(n);
  c2.reserve(n);
  f2.reserve(p.features.size());
  p.segs.clear();
  for (int v = 0; v < 256; ++v) {
    std::vector<size_t> idx;
    for (size_t q = 0; q < n; ++q)
      if (p.meta[q].var == v) idx.push_back(q);
    if (idx.empty()) continue;
    Segment g;
    g.variant = v;
    g.begin = int32_t(items.size());
    int64_t maxc = 0;
    const auto bins = deal(p, idx, cost);
    for (int x = 0; x < kXcds; ++x) {
      g.xcd_begin[x] = int32_t(items.size()) - g.begin;
      for (size_t q : bins[size_t(x)]) {
        items.push_back(p.items[q]);
        metas.push_back(p.meta[q]);
        c2.push_back(cost[q]);
        for (int f = 0; f < 5; ++f) f2.push_back(p.features[q * 5 + size_t(f)]);
      }
      maxc = std::max<int64_t>(maxc, int64_t(bins[size_t(x)].size()));
    }
    g.xcd_begin[kXcds] = int32_t(items.size()) - g.begin;
    g.end = int32_t(items.size());
    g.grid = maxc * kXcds;
    p.segs.push_back(g);
  }
  p.items.swap(items);
  p.meta.swap(metas);
  p.cost.swap(c2);
  p.features.swap(f2);
  if (p.dev_klists) batch_device_klists(p);
}

void cut_items(HostPlan& p, int variant) {
  int cv[kSizeClasses];
  for (int c = 0; c < kSizeClasses; ++c) cv[c] = variant;
  cut_items(p, cv);
}

void cut_items(HostPlan& p, const int class_var[kSizeClasses]) {
  const bool bf16 = p.cfg.precision == 2;
  std::vector<std::pair<int, int>> rs, cs;
  p.items.clear();
  p.meta.clear();
  p.features.clear();
  for (int c = 0; c < kSizeClasses; ++c) p.class_var[c] = class_var[c];
  for (const CBlock& cb : p.cblocks) {
    const int variant = class_var[size_class(cb.m, cb.n)];
    const Variant& var = bf16 ? kBf16Variants[variant] : kVariants[variant];
    cut_dim(cb.m, var.tm / 16, rs);
    cut_dim(cb.n, var.tn / 16, cs);
    for (auto& r : rs)
      for (auto& c : cs) {
        Item it;
        it.c_off = cb.c_off;
        it.tri_begin = cb.tri_begin;
        it.tri_count = cb.tri_count;
        it.r0 = uint16_t(r.first);
        it.h = uint16_t(r.second);
        it.c0 = uint16_t(c.first);
        it.w = uint16_t(c.second);
        it.ldc = uint16_t(cb.n);
        it.ldm = uint16_t(cb.m);
        it.product = 0;
        p.items.push_back(it);
        p.meta.push_back(ItemMeta{cb.ci, cb.cj, variant, cb.sk});
        p.features.push_back(std::log(float(it.h)));
        p.features.push_back(std::log(float(it.w)));
        p.features.push_back(std::log(float(std::max(1.0, cb.sk))));
        p.features.push_back(std::log(float(std::max<uint32_t>(1, cb.tri_count))));
        p.features.push_back(float(p.k_total > 0 ? cb.sk / p.k_total : 0.0));
      }
  }
  if (p.ksplit > 1) {
    // reduction variant: each task's k-list cut into up to ksplit contiguous pieces of equal
    // triple count; piece s writes its partial sums into partial buffer s (the task's product)
    std::vector<Item> its;
    std::vector<ItemMeta> ms;
    std::vector<float> fs;
    for (size_t q = 0; q < p.items.size(); ++q) {
      const Item& it = p.items[q];
      const uint64_t T = it.tri_count;
      const uint64_t S = std::min<uint64_t>(uint64_t(p.ksplit), std::max<uint64_t>(T, 1));
      for (uint64_t s = 0; s < S; ++s) {
        Item x = it;
        const uint64_t b0 = T * s / S, b1 = T * (s + 1) / S;
        x.tri_begin = uint32_t(it.tri_begin + b0);
        x.tri_count = uint32_t(b1 - b0);
        x.product = uint32_t(s);
        its.push_back(x);
        ms.push_back(p.meta[q]);
        for (int f = 0; f < 5; ++f) fs.push_back(p.features[q * 5 + size_t(f)]);
      }
    }
    p.items.swap(its);
    p.meta.swap(ms);
    p.features.swap(fs);
  }
}

// Complex elements: the product runs as the real product of the embeddings
//   op(A)_ik -> [[Re, -Im], [Im, Re]] (2 r_i x 2 s_k),  op(B)_kj -> [Re; Im] (2 s_k x t_j),
// whose C block is [Re C_ij; Im C_ij] (2 r_i x t_j), planned like any real product over the
// doubled row and inner tilings; the tables of the embedding pass and of the epilogue are added.
static std::string build_complex_plan(HostPlan& p, int64_t M, const int64_t* rows, int64_t K,
                                      const int64_t* inner, int64_t N, const int64_t* cols,
                                      const uint64_t* a_bits, const uint64_t* b_bits,
                                      const PlanConfig& cfg, int* code) {
  std::string e;
  if (cfg.cplx != 1) return "elem must be 0 (real) or 1 (complex)";
  if (!(e = check_tiling("row_sizes", M, rows)).empty()) return e;
  if (!(e = check_tiling("inner_sizes", K, inner)).empty()) return e;
  if (!(e = check_tiling("col_sizes", N, cols)).empty()) return e;
  for (int64_t i = 0; i < M; ++i)
    if (rows[i] > kMaxBlock / 2) return "row_sizes: complex blocks allow at most 32767 rows";
  for (int64_t k = 0; k < K; ++k)
    if (inner[k] > kMaxBlock / 2) return "inner_sizes: complex blocks allow at most 32767 inner";
  if (cfg.trans_a < 0 || cfg.trans_a > 2 || cfg.trans_b < 0 || cfg.trans_b > 2)
    return "trans_a and trans_b must be 0, 1 or 2";
  const int oa = cfg.trans_a, ob = cfg.trans_b;
  if (!(e = check_bits("a_bits", oa ? K : M, oa ? M : K, a_bits)).empty()) return e;
  if (!(e = check_bits("b_bits", ob ? N : K, ob ? K : N, b_bits)).empty()) return e;
  const int64_t wk = words_for(K), wn = words_for(N);
  std::vector<uint64_t> la = oa ? transpose_bits(a_bits, K, M)
                                : std::vector<uint64_t>(a_bits, a_bits + M * wk);
  std::vector<uint64_t> lb = ob ? transpose_bits(b_bits, N, K)
                                : std::vector<uint64_t>(b_bits, b_bits + K * wn);
  std::vector<int64_t> r2(rows, rows + M), s2(inner, inner + K);
  for (auto& x : r2) x *= 2;
  for (auto& x : s2) x *= 2;
  PlanConfig rc = cfg;
  rc.cplx = 0;
  rc.trans_a = rc.trans_b = 0;
  rc.out_f32 = 0;  // the real product writes FP64 [Re; Im] blocks; the epilogue rounds
  e = build_plan(p, M, r2.data(), K, s2.data(), N, cols, la.data(), lb.data(), rc, code);
  if (!e.empty()) return e;
  *code = BSM_E_INVALID;
  p.cplx = 1;
  p.zop_a = oa;
  p.zop_b = ob;
  p.z_out_f32 = cfg.out_f32;
  p.cfg.cplx = 1;
  // the caller's packed offsets (complex elements) of the stored blocks
  std::vector<int64_t> st_a, st_b;
  int64_t nb;
  {
    std::vector<int64_t> r1(rows, rows + M), s1(inner, inner + K), t1(cols, cols + N);
    std::vector<uint64_t> sa(a_bits, a_bits + (oa ? K * words_for(M) : M * wk));
    std::vector<uint64_t> sb(b_bits, b_bits + (ob ? N * wk : K * wn));
    if (oa) pack_offsets(K, M, s1, r1, sa, st_a, nb);
    else pack_offsets(M, K, r1, s1, sa, st_a, nb);
    if (ob) pack_offsets(N, K, t1, s1, sb, st_b, nb);
    else pack_offsets(K, N, s1, t1, sb, st_b, nb);
  }
  const int ma = (oa ? kZTrans : 0) | (oa == 2 ? kZConj : 0);
  const int mb = kZRight | (ob ? kZTrans : 0) | (ob == 2 ? kZConj : 0);
  for (int64_t i = 0; i < M; ++i)
    for (int64_t k = 0; k < K; ++k) {
      const int64_t o = p.a_off[size_t(i * K + k)];
      if (o < 0) continue;
      const int64_t so = oa ? st_a[size_t(k * M + i)] : st_a[size_t(i * K + k)];
      const int64_t R = rows[i], W = inner[k];  // embedded as 2R x 2W
      for (int64_t x = 0; x < R; x += kZBand)
        p.zembed_a.push_back(ZBlock{so + (oa ? x : x * W), o + x * 2 * W,
                                    int32_t(std::min<int64_t>(kZBand, R - x)), int32_t(W), ma, int32_t(R)});
    }
  for (int64_t k = 0; k < K; ++k)
    for (int64_t j = 0; j < N; ++j) {
      const int64_t o = p.b_off[size_t(k * N + j)];
      if (o < 0) continue;
      const int64_t so = ob ? st_b[size_t(j * K + k)] : st_b[size_t(k * N + j)];
      const int64_t R = inner[k], W = cols[j];  // embedded as 2R x W
      for (int64_t x = 0; x < R; x += kZBand)
        p.zembed_b.push_back(ZBlock{so + (ob ? x : x * W), o + x * W,
                                    int32_t(std::min<int64_t>(kZBand, R - x)), int32_t(W), mb, int32_t(R)});
    }
  for (int64_t i = 0; i < M; ++i)
    for (int64_t j = 0; j < N; ++j) {
      const int64_t o = p.c_off[size_t(i * N + j)];
      if (o < 0) continue;
      const int64_t n = rows[i] * cols[j];
      for (int64_t e = 0; e < n; e += kZCPiece)
        p.zc.push_back(ZCBlock{o / 2, n, e, std::min(n, e + kZCPiece)});
    }
  *code = BSM_OK;
  return "";
}

std::string build_plan(HostPlan& p, int64_t M, const int64_t* rows, int64_t K,
                       const int64_t* inner, int64_t N, const int64_t* cols,
                       const uint64_t* a_bits, const uint64_t* b_bits, const PlanConfig& cfg,
                       int* code) {
  *code = BSM_E_INVALID;
  std::string e;
  if (cfg.cplx) return build_complex_plan(p, M, rows, K, inner, N, cols, a_bits, b_bits, cfg, code);
  if (!(e = check_tiling("row_sizes", M, rows)).empty()) return e;
  if (!(e = check_tiling("inner_sizes", K, inner)).empty()) return e;
  if (!(e = check_tiling("col_sizes", N, cols)).empty()) return e;
  if (cfg.trans_a < 0 || cfg.trans_a > 1 || cfg.trans_b < 0 || cfg.trans_b > 1)
    return "trans_a and trans_b must be 0 or 1";
  const bool ta = cfg.trans_a != 0, tb = cfg.trans_b != 0;
  // a transposed operand's shape is given as stored: K x M for A, N x K for B
  if (!(e = check_bits("a_bits", ta ? K : M, ta ? M : K, a_bits)).empty()) return e;
  if (!(e = check_bits("b_bits", tb ? N : K, tb ? K : N, b_bits)).empty()) return e;
  if (cfg.precision < 0 || cfg.precision > 2) return "unknown precision";
  if (cfg.sched < 0 || cfg.sched > 1) return "unknown scheduler";
  if (cfg.k_window < 0) return "negative k_window";
  if (cfg.tile < 0 || cfg.tile > (cfg.precision == 2 ? kNumBf16Variants : kNumVariants))
    return "unknown tile variant";
  if (cfg.order < ORDER_LOCALITY || cfg.order > ORDER_AUTO) return "unknown task order";
  if (cfg.device_klists < -1) return "device_klists must be -1, 0, 1 or a batch size >= 2";
  if (cfg.k_split < -1 || cfg.k_split > 16) return "k_split must be -1 (auto), 0, 1 or 2..16";
  if (cfg.patch_r < 1 || cfg.patch_c < 1) return "patch sizes must be >= 1";

  p.cfg = cfg;
  p.M = M; p.K = K; p.N = N;
  p.rows.assign(rows, rows + M);
  p.inner.assign(inner, inner + K);
  p.cols.assign(cols, cols + N);
  int64_t wk = words_for(K), wn = words_for(N);
  // the shapes of op(A) and op(B), which everything below works on
  if (ta) p.a_bits = transpose_bits(a_bits, K, M);
  else p.a_bits.assign(a_bits, a_bits + M * wk);
  if (tb) p.b_bits = transpose_bits(b_bits, N, K);
  else p.b_bits.assign(b_bits, b_bits + K * wn);

  // S1: packed offsets of op(A) and op(B) in the product's layout, and for a transposed operand
  // the offsets of its blocks as stored (st_a[k M + i] of A_ki = op(A)_ik, st_b[j K + k])
  p.a_elems = pack_offsets(M, K, p.rows, p.inner, p.a_bits, p.a_off, p.a_blocks);
  p.b_elems = pack_offsets(K, N, p.inner, p.cols, p.b_bits, p.b_off, p.b_blocks);
  std::vector<int64_t> st_a, st_b;
  if (ta) {
    int64_t nb;
    std::vector<uint64_t> sb(a_bits, a_bits + K * words_for(M));
    pack_offsets(K, M, p.inner, p.rows, sb, st_a, nb);
  }
  if (tb) {
    int64_t nb;
    std::vector<uint64_t> sb(b_bits, b_bits + N * wk);
    pack_offsets(N, K, p.cols, p.inner, sb, st_b, nb);
  }

  // S2: C-shape, row i = OR of B's rows k over A's present (i, k)
  p.c_bits.assign(size_t(M * wn), 0);
  for (int64_t i = 0; i < M; ++i) {
    uint64_t* crow = p.c_bits.data() + i * wn;
    for (int64_t w = 0; w < wk; ++w) {
      uint64_t x = p.a_bits[size_t(i * wk + w)];
      while (x) {
        int64_t k = w * 64 + __builtin_ctzll(x);
        x &= x - 1;
        const uint64_t* brow = p.b_bits.data() + k * wn;
        for (int64_t v = 0; v < wn; ++v) crow[v] |= brow[v];
      }
    }
  }
  p.c_elems = pack_offsets(M, N, p.rows, p.cols, p.c_bits, p.c_off, p.c_blocks);
  if (p.a_elems >= kMaxElems || p.b_elems >= kMaxElems || p.c_elems >= kMaxElems) {
    *code = BSM_E_NOMEM;
    return "a tile buffer exceeds 2^48 elements";
  }

  // split-bf16 form: operand blocks in the slice planes (inner size padded to 32; B transposed)
  std::vector<int64_t> a_off32, b_off32;
  const bool bf16 = cfg.precision == 2;
  if (bf16) {
    a_off32.assign(p.a_off.size(), -1);
    b_off32.assign(p.b_off.size(), -1);
    int64_t pos = 0;
    for (int64_t i = 0; i < M; ++i)
      for (int64_t k = 0; k < K; ++k) {
        int64_t o = p.a_off[size_t(i * K + k)];
        if (o < 0) continue;
        a_off32[size_t(i * K + k)] = pos;
        // stored as r_i x s_k, or (transposed) as s_k x r_i
        if (ta)
          push_split(p.split_a, st_a[size_t(k * M + i)], pos, p.rows[size_t(i)], p.inner[size_t(k)],
                     p.rows[size_t(i)], 1);
        else
          push_split(p.split_a, o, pos, p.rows[size_t(i)], p.inner[size_t(k)], p.inner[size_t(k)], 0);
        pos += p.rows[size_t(i)] * pad_k(p.inner[size_t(k)]);
      }
    p.a_elems32 = pos;
    pos = 0;
    for (int64_t k = 0; k < K; ++k)
      for (int64_t j = 0; j < N; ++j) {
        int64_t o = p.b_off[size_t(k * N + j)];
        if (o < 0) continue;
        b_off32[size_t(k * N + j)] = pos;
        // stored as s_k x t_j (written transposed), or (transposed) as t_j x s_k
        if (tb)
          push_split(p.split_b, st_b[size_t(j * K + k)], pos, p.cols[size_t(j)], p.inner[size_t(k)],
                     p.inner[size_t(k)], 0);
        else
          push_split(p.split_b, o, pos, p.cols[size_t(j)], p.inner[size_t(k)], p.cols[size_t(j)], 1);
        pos += p.cols[size_t(j)] * pad_k(p.inner[size_t(k)]);
      }
    p.b_elems32 = pos;
    if (p.a_elems32 >= kMaxElems / 4 || p.b_elems32 >= kMaxElems / 4) {
      *code = BSM_E_NOMEM;
      return "slice planes exceed the descriptor range";
    }
  } else {
    // FP64 / FP32 forms: a transposed operand is written into the product's layout by a
    // transposition pass (stored block rows x cols -> cols x rows), block by block
    if (ta)
      for (int64_t i = 0; i < M; ++i)
        for (int64_t k = 0; k < K; ++k) {
          const int64_t o = p.a_off[size_t(i * K + k)];
          if (o >= 0)
            push_transpose(p.xpose_a, st_a[size_t(k * M + i)], o, int32_t(p.inner[size_t(k)]),
                           int32_t(p.rows[size_t(i)]));
        }
    if (tb)
      for (int64_t k = 0; k < K; ++k)
        for (int64_t j = 0; j < N; ++j) {
          const int64_t o = p.b_off[size_t(k * N + j)];
          if (o >= 0)
            push_transpose(p.xpose_b, st_b[size_t(j * K + k)], o, int32_t(p.cols[size_t(j)]),
                           int32_t(p.inner[size_t(k)]));
        }
  }

  // S3: k-lists (A row AND B column) and tasks.  First, per present C block, the k-list's length
  // and summed inner size, counted from the bitmap words (block rows in parallel); then either
  // the triples themselves in a host list, or, when they would not fit it, the tables from which
  // the device builds them batch by batch.
  std::vector<uint64_t> bt(size_t(N * wk), 0);  // B's shape transposed: column j's k bits
  for (int64_t k = 0; k < K; ++k)
    for (int64_t j = 0; j < N; ++j)
      if (test_bit(p.b_bits.data(), wn, k, j)) bt[size_t(j * wk + (k >> 6))] |= uint64_t(1) << (k & 63);
  std::vector<int64_t> crow(size_t(M) + 1, 0);  // present C blocks before block row i
  for (int64_t i = 0; i < M; ++i) {
    int64_t c = 0;
    for (int64_t v = 0; v < wn; ++v) c += __builtin_popcountll(p.c_bits[size_t(i * wn + v)]);
    crow[size_t(i) + 1] = crow[size_t(i)] + c;
  }
  std::vector<uint32_t> cnt(size_t(crow[size_t(M)]));
  std::vector<double> sks(size_t(crow[size_t(M)]));
  // inner sizes grouped into per-size k masks when there are few distinct sizes (the summed
  // inner size is then a handful of masked popcounts instead of a walk over the bits)
  std::map<int64_t, std::vector<uint64_t>> size_mask;
  for (int64_t k = 0; k < K && size_mask.size() <= 16; ++k) {
    auto& m = size_mask[p.inner[size_t(k)]];
    if (m.empty()) m.assign(size_t(wk), 0);
    m[size_t(k >> 6)] |= uint64_t(1) << (k & 63);
  }
  const bool by_mask = size_mask.size() <= 16;
  auto count_rows = [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      int64_t q = crow[size_t(i)];
      for (int64_t j = 0; j < N; ++j) {
        if (!test_bit(p.c_bits.data(), wn, i, j)) continue;
        const uint64_t* ar = p.a_bits.data() + i * wk;
        const uint64_t* br = bt.data() + j * wk;
        uint32_t c = 0;
        double sk = 0;
        if (by_mask) {
          for (int64_t w = 0; w < wk; ++w) c += uint32_t(__builtin_popcountll(ar[w] & br[w]));
          for (const auto& sm : size_mask) {
            int64_t n = 0;
            for (int64_t w = 0; w < wk; ++w) n += __builtin_popcountll(ar[w] & br[w] & sm.second[size_t(w)]);
            sk += double(sm.first) * double(n);
          }
        } else {
          for (int64_t w = 0; w < wk; ++w) {
            uint64_t x = ar[w] & br[w];
            while (x) {
              const int64_t k = w * 64 + __builtin_ctzll(x);
              x &= x - 1;
              ++c;
              sk += double(p.inner[size_t(k)]);
            }
          }
        }
        cnt[size_t(q)] = c;
        sks[size_t(q)] = sk;
        ++q;
      }
    }
  };
  {
    const int64_t nthreads = std::max<int64_t>(1, std::min<int64_t>(
        std::min<int64_t>(16, int64_t(std::thread::hardware_concurrency())), (M * N) / 4096 + 1));
    std::vector<std::thread> pool;
    for (int64_t t = 0; t < nthreads; ++t)
      pool.emplace_back(count_rows, M * t / nthreads, M * (t + 1) / nthreads);
    for (auto& th : pool) th.join();
  }
  int64_t total = 0;
  for (uint32_t c : cnt) total += c;
  p.triples_total = total;
  p.dev_klists = cfg.device_klists > 0 || (cfg.device_klists == 0 && total > kHostTriples);
  if (!p.dev_klists && total >= (int64_t(1) << 32)) {
    *code = BSM_E_NOMEM;
    return "more than 2^32 block triples for a host list (device k-lists were turned off)";
  }
  p.tri.clear();
  p.items.clear();
  p.features.clear();
  p.useful_flops = 0;
  p.cblocks.clear();
  p.cblocks.reserve(cnt.size());
  if (!p.dev_klists) p.tri.reserve(size_t(total));
  for (int64_t i = 0; i < M; ++i) {
    int64_t q = crow[size_t(i)];
    for (int64_t j = 0; j < N; ++j) {
      int64_t co = p.c_off[size_t(i * N + j)];
      if (co < 0) continue;
      const size_t tb = p.dev_klists ? 0 : p.tri.size();
      if (!p.dev_klists) {
        for (int64_t w = 0; w < wk; ++w) {
          uint64_t x = p.a_bits[size_t(i * wk + w)] & bt[size_t(j * wk + w)];
          while (x) {
            int64_t k = w * 64 + __builtin_ctzll(x);
            x &= x - 1;
            Triple t;
            const int64_t ao = bf16 ? a_off32[size_t(i * K + k)] : p.a_off[size_t(i * K + k)];
            const int64_t bo = bf16 ? b_off32[size_t(k * N + j)] : p.b_off[size_t(k * N + j)];
            t.a = uint64_t(ao) | (uint64_t(p.inner[size_t(k)]) << 48);
            t.b = uint64_t(bo) | (uint64_t(k) << 48);
            p.tri.push_back(t);
          }
        }
      }
      const double sk = sks[size_t(q)];
      const uint32_t tc = cnt[size_t(q)];
      ++q;
      int m = int(p.rows[size_t(i)]), n = int(p.cols[size_t(j)]);
      p.useful_flops += 2.0 * m * n * sk;
      p.cblocks.push_back(CBlock{co, uint32_t(tb), tc, m, n, int32_t(i), int32_t(j), sk});
    }
  }
  if (p.dev_klists) {
    // the device's tables: A offsets by (i, k), B offsets by (j, k), both in the form's layout
    p.wk = wk;
    p.bt_bits.swap(bt);
    p.a_tab.assign(size_t(M * K), -1);
    p.bt_tab.assign(size_t(N * K), -1);
    for (int64_t i = 0; i < M; ++i)
      for (int64_t k = 0; k < K; ++k)
        p.a_tab[size_t(i * K + k)] = bf16 ? a_off32[size_t(i * K + k)] : p.a_off[size_t(i * K + k)];
    for (int64_t k = 0; k < K; ++k)
      for (int64_t j = 0; j < N; ++j)
        p.bt_tab[size_t(j * K + k)] = bf16 ? b_off32[size_t(k * N + j)] : p.b_off[size_t(k * N + j)];
  }
  p.k_total = 0;
  for (int64_t k = 0; k < K; ++k) p.k_total += double(p.inner[size_t(k)]);
  cut_items(p, cfg.tile > 0 ? cfg.tile - 1 : (bf16 ? kDefaultBf16Variant : kDefaultVariant));
  // reduction variant (Sec. 3.2 splits every update into a multiply task and a reduction into C;
  // the tile kernel fuses the two, which leaves a product with few C tiles too few tasks): cut
  // every task's k-list into pieces whose partial sums a reduction pass adds, in piece order
  if (cfg.k_split > 1 || cfg.k_split == -1) {
    const bool windows = cfg.k_window != 0 && cfg.k_window < K;
    if (p.dev_klists || windows) {
      if (cfg.k_split > 1) {
        *code = BSM_E_UNSUPPORTED;
        return "k_split needs k-lists in the host list and k_window 0";
      }
    } else {
      int S = cfg.k_split;
      if (S == -1) {  // auto: split only products with fewer than 1024 tasks, towards 2048
        const int64_t n = int64_t(p.items.size());
        S = n > 0 && n < 1024 ? int(std::min<int64_t>(16, (2048 + n - 1) / n)) : 1;
      }
      if (S > 1) {
        p.ksplit = S;
        cut_items(p, p.class_var);
      }
    }
  }
  // S5: k-windows (0 = all K inner blocks in flight at once)
  p.k_window_eff = (cfg.k_window == 0 || cfg.k_window >= K) ? std::max<int64_t>(K, 1) : cfg.k_window;
  p.windows = K > 0 ? (K + p.k_window_eff - 1) / p.k_window_eff : 1;
  // S4: cost and order
  schedule(p, flop_costs(p));
  *code = BSM_OK;
  return "";
}

std::string merge_plans(HostPlan& out, const std::vector<const HostPlan*>& parts, int* code) {
  *code = BSM_E_MISMATCH;
  if (parts.empty()) {
    *code = BSM_E_INVALID;
    return "empty batch";
  }
  const HostPlan& p0 = *parts[0];
  out = HostPlan();
  out.cfg = p0.cfg;
  for (int c = 0; c < kSizeClasses; ++c) out.class_var[c] = p0.class_var[c];
  out.windows = 1;
  out.k_window_eff = 1;
  for (size_t q = 0; q < parts.size(); ++q) {
    const HostPlan& p = *parts[q];
    if (p.cfg.precision != p0.cfg.precision) return "batch members differ in precision";
    if (p.windows != 1) return "batch members must issue all k-iterations at once (k_window 0)";
    if (p.ksplit > 1) {
      *code = BSM_E_UNSUPPORTED;
      return "batch members cannot split their k-lists (k_split)";
    }
    if (p.dev_klists) {
      *code = BSM_E_UNSUPPORTED;
      return "batch members must keep their k-lists on the host (device k-lists are per plan)";
    }
    const uint64_t tb = out.tri.size();
    if (tb + p.tri.size() >= (uint64_t(1) << 32)) {
      *code = BSM_E_NOMEM;
      return "more than 2^32 block triples in the batch";
    }
    out.tri.insert(out.tri.end(), p.tri.begin(), p.tri.end());
    for (const Item& it0 : p.items) {
      Item it = it0;
      it.tri_begin = uint32_t(it.tri_begin + tb);
      it.product = uint32_t(q);
      out.items.push_back(it);
    }
    out.meta.insert(out.meta.end(), p.meta.begin(), p.meta.end());
    out.features.insert(out.features.end(), p.features.begin(), p.features.end());
    out.useful_flops += p.useful_flops;
    out.c_blocks += p.c_blocks;
  }
  schedule(out, flop_costs(out));
  *code = BSM_OK;
  return "";
}

}  // namespace bsm
