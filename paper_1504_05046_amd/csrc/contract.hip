// Block-sparse tensor contraction (the paper's title and Sec. 1: the block-sparse matrix product
// as a step towards block-sparse tensor computing) as permute + block-sparse multiply:
//
//   C[free_A, free_B] = alpha sum_{contracted} A[...] B[...] (+ C)
//
// A is matricized with its free modes (in C's order) as the row index and the contracted modes
// (in A's order) as the inner index; B with the contracted modes (same order) as the inner index
// and its free modes (in C's order) as the column index.  Row, inner and column blocks are tuples
// of mode blocks (mixed radix, last mode fastest) whose sizes are products of the modes' block
// sizes, so the matricized operands are block-sparse matrices with nonuniform blocks and the
// product is an ordinary plan of this library.  A permutation pass brings an operand into matrix
// order unless its mode order already is (then it is used in place), and one brings C back into
// its own mode order unless C lists A's free modes before B's.  A block whose modes stay in order
// is copied, one whose modes fall into two swapped groups is transposed through LDS, any other is
// permuted element by element; each in pieces of one workgroup.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/bsm.h"
#include "errors.hpp"
#include "kernels.hpp"
#include "staging.hpp"

using namespace bsm;

#define TC_HIP(call, what)                                                                  \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return set_error(BSM_E_HIP, std::string(what) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace {

// A validated copy of a tensor descriptor.
struct Tensor {
  int order = 0;
  std::vector<int32_t> modes;
  std::vector<int64_t> nb;                  // blocks per mode
  std::vector<std::vector<int64_t>> sizes;  // block sizes per mode
  std::vector<uint64_t> bits;               // block shape over the flattened grid
  int64_t grid = 1;                         // blocks in the grid
  bool present(int64_t q) const { return (bits[size_t(q / 64)] >> (q % 64)) & 1; }
  // mode block indices of flattened block q (row-major, last mode fastest)
  void decode(int64_t q, int64_t* idx) const {
    for (int m = order - 1; m >= 0; --m) {
      idx[m] = q % nb[size_t(m)];
      q /= nb[size_t(m)];
    }
  }
  int pos(int32_t label) const {
    for (int m = 0; m < order; ++m)
      if (modes[size_t(m)] == label) return m;
    return -1;
  }
};

std::string load_tensor(const char* name, const bsm_tensor* d, Tensor& t) {
  const std::string n(name);
  if (!d) return n + " is null";
  if (d->order < 1 || d->order > kMaxModes) return n + ": order must be 1..8";
  if (!d->modes || !d->nblocks) return n + ": null mode or block-count vector";
  t.order = d->order;
  t.modes.assign(d->modes, d->modes + d->order);
  t.nb.assign(d->nblocks, d->nblocks + d->order);
  int64_t nsizes = 0;
  for (int m = 0; m < t.order; ++m) {
    for (int x = 0; x < m; ++x)
      if (t.modes[size_t(x)] == t.modes[size_t(m)]) return n + ": a label appears twice";
    if (t.nb[size_t(m)] < 0) return n + ": negative block count";
    if (t.nb[size_t(m)] > 0 && t.grid > (int64_t(1) << 40) / t.nb[size_t(m)])
      return n + ": block grid above 2^40 blocks";
    t.grid *= t.nb[size_t(m)];
    nsizes += t.nb[size_t(m)];
  }
  if (nsizes && !d->sizes) return n + ": null size vector";
  const int64_t* s = d->sizes;
  for (int m = 0; m < t.order; ++m) {
    t.sizes.emplace_back(s, s + t.nb[size_t(m)]);
    for (int64_t v : t.sizes.back())
      if (v < 1 || v > 65535) return n + ": block size outside [1, 65535]";
    s += t.nb[size_t(m)];
  }
  const int64_t words = (t.grid + 63) / 64;
  if (words && !d->bits) return n + ": null bitmap";
  t.bits.assign(d->bits, d->bits + words);
  if (t.grid % 64 && words && (t.bits.back() & (~uint64_t(0) << (t.grid % 64))))
    return n + ": padding bit set";
  return "";
}

// Mixed-radix index of the tuple idx[pos[0..]] over the radices nb[pos[..]].
int64_t tuple_index(const std::vector<int>& pos, const int64_t* idx, const Tensor& t) {
  int64_t r = 0;
  for (int p : pos) r = r * t.nb[size_t(p)] + idx[p];
  return r;
}

}  // namespace

// A permutation pass split by kind: blocks whose modes stay in order are copies, blocks whose
// modes fall into two swapped groups are 2-D transposes, the rest go element by element.
struct Pass {
  std::vector<CopyBlock> copy;
  std::vector<XposeBlock> xpose;
  std::vector<PermBlock> perm;
  CopyBlock* d_copy = nullptr;
  XposeBlock* d_xpose = nullptr;
  PermBlock* d_perm = nullptr;
  bool empty() const { return copy.empty() && xpose.empty() && perm.empty(); }
};

// Cut a whole-block permutation into pieces of one workgroup.  Source modes m and m+1 that stay
// adjacent in the destination (stride[m] = stride[m+1] ext[m+1]) merge into one group, modes of
// extent 1 drop out; one group is a copy, two groups in swapped order a transpose.
static void lower(const PermBlock& b, bool generic_only, Pass& out) {
  int64_t n = 1;
  for (int m = 0; m < b.order; ++m) n *= b.ext[m];
  if (n == 0) return;
  if (!generic_only) {
    std::vector<std::pair<int64_t, int64_t>> g;  // (extent, destination stride), source order
    for (int m = 0; m < b.order; ++m) {
      if (b.ext[m] == 1) continue;
      if (!g.empty() && g.back().second == b.dst_stride[m] * b.ext[m]) {
        g.back().first *= b.ext[m];
        g.back().second = b.dst_stride[m];
      } else {
        g.emplace_back(b.ext[m], b.dst_stride[m]);
      }
    }
    if (g.empty() || (g.size() == 1 && g[0].second == 1)) {
      push_copy(out.copy, b.src_off, b.dst_off, n);
      return;
    }
    if (g.size() == 2 && g[1].second == g[0].first && g[0].second == 1 && g[0].first <= 65535 &&
        g[1].first <= 65535) {
      push_transpose(out.xpose, b.src_off, b.dst_off, int32_t(g[0].first), int32_t(g[1].first));
      return;
    }
  }
  for (int64_t e = 0; e < n; e += kPermPiece) {
    PermBlock piece = b;
    piece.e0 = e;
    piece.e1 = std::min(n, e + kPermPiece);
    out.perm.push_back(piece);
  }
}

struct bsm_tc_plan {
  bsm_plan* mat = nullptr;
  bsm_tc_info info{};
  std::vector<PermBlock> pa, pb, pc;  // whole blocks
  Pass xa, xb, xc;                    // the pieces launched
  int64_t a_mat = 0, b_mat = 0, c_mat = 0;  // elements of the matricized operands
  int c_f32 = 0;
  std::vector<uint64_t> c_bits;
  double* d_A = nullptr;
  double* d_B = nullptr;
  double* d_C = nullptr;
  bool ready = false;
};

static void tc_free(bsm_tc_plan* p) {
  if (p->mat) bsm_plan_destroy(p->mat);
  // also the buffers of a preparation that failed part-way
  std::vector<void*> bufs = {p->d_A, p->d_B, p->d_C};
  for (Pass* x : {&p->xa, &p->xb, &p->xc})
    for (void* ptr : {static_cast<void*>(x->d_copy), static_cast<void*>(x->d_xpose),
                      static_cast<void*>(x->d_perm)})
      bufs.push_back(ptr);
  bool any = false;
  for (void* ptr : bufs) any = any || ptr;
  if (any) {
    (void)hipDeviceSynchronize();
    for (void* ptr : bufs)
      if (ptr) (void)hipFree(ptr);
  }
  delete p;
}

static bsm_status upload_pass(Pass& x) {
  auto up = [](auto** dst, const auto& v) -> bsm_status {
    const size_t bytes = v.size() * sizeof(v[0]);
    if (!bytes) return BSM_OK;
    TC_HIP(hipMalloc(dst, bytes), "hipMalloc(permutation tables)");
    TC_HIP(hipMemcpy(*dst, v.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy(permutation tables)");
    return BSM_OK;
  };
  bsm_status st;
  if ((st = up(&x.d_copy, x.copy)) != BSM_OK) return st;
  if ((st = up(&x.d_xpose, x.xpose)) != BSM_OK) return st;
  return up(&x.d_perm, x.perm);
}

static bsm_status run_pass(const Pass& x, const double* src, void* dst, int c_f32, int accumulate,
                           hipStream_t s, const char* what) {
  if (!x.copy.empty())
    TC_HIP(launch_copy_blocks(x.d_copy, int64_t(x.copy.size()), src, static_cast<double*>(dst), s), what);
  if (!x.xpose.empty())
    TC_HIP(launch_transpose_f64(x.d_xpose, int64_t(x.xpose.size()), src, static_cast<double*>(dst), s),
           what);
  if (!x.perm.empty())
    TC_HIP(launch_permute_blocks(x.d_perm, int64_t(x.perm.size()), src, dst, c_f32, accumulate, s),
           what);
  return BSM_OK;
}

// Destination strides, per source mode, of a row-major layout over `layout` (source mode
// positions, outermost first) with the source block's extents ext.
static void strides_for(const std::vector<int>& layout, const int32_t* ext, int64_t* stride) {
  int64_t s = 1;
  for (size_t x = layout.size(); x-- > 0;) {
    stride[layout[x]] = s;
    s *= ext[layout[x]];
  }
}

// Matricization of one operand: its present blocks in matrix order with their matrix offsets,
// and the permutation table (source = the operand's packed blocks).
static void matricize(const Tensor& t, const std::vector<int>& rows, const std::vector<int>& cols,
                      int64_t ncols, std::vector<uint64_t>& mbits, int64_t& melems,
                      std::vector<PermBlock>& table, int64_t& telems) {
  struct Blk { int64_t key, src, n; int64_t idx[kMaxModes]; };
  std::vector<Blk> blks;
  int64_t src = 0;
  const int64_t wc = (ncols + 63) / 64;
  for (int64_t q = 0; q < t.grid; ++q) {
    if (!t.present(q)) continue;
    Blk b{};
    t.decode(q, b.idx);
    b.n = 1;
    for (int m = 0; m < t.order; ++m) b.n *= t.sizes[size_t(m)][size_t(b.idx[m])];
    const int64_t r = tuple_index(rows, b.idx, t), c = tuple_index(cols, b.idx, t);
    b.key = r * ncols + c;
    b.src = src;
    src += b.n;
    mbits[size_t(r * wc + c / 64)] |= uint64_t(1) << (c % 64);
    blks.push_back(b);
  }
  telems = src;
  std::sort(blks.begin(), blks.end(), [](const Blk& x, const Blk& y) { return x.key < y.key; });
  std::vector<int> layout(rows);
  layout.insert(layout.end(), cols.begin(), cols.end());
  int64_t dst = 0;
  for (const Blk& b : blks) {
    PermBlock pbk{};
    pbk.src_off = b.src;
    pbk.dst_off = dst;
    pbk.order = t.order;
    for (int m = 0; m < t.order; ++m) pbk.ext[m] = int32_t(t.sizes[size_t(m)][size_t(b.idx[m])]);
    strides_for(layout, pbk.ext, pbk.dst_stride);
    table.push_back(pbk);
    dst += b.n;
  }
  melems = dst;
}

extern "C" {

bsm_status bsm_tc_plan_create(bsm_tc_plan** out, const bsm_tensor* A, const bsm_tensor* B,
                              int32_t c_order, const int32_t* c_modes, const bsm_options* opt) {
  if (!out) return set_error(BSM_E_INVALID, "out is null");
  *out = nullptr;
  bsm_options o;
  bsm_options_default(&o);
  if (opt) o = *opt;
  if (o.elem != BSM_REAL) return set_error(BSM_E_UNSUPPORTED, "contractions take real tensors");
  if (o.trans_a || o.trans_b)
    return set_error(BSM_E_UNSUPPORTED, "contractions express transposes by their mode labels");
  Tensor ta, tb;
  std::string err;
  if (!(err = load_tensor("A", A, ta)).empty()) return set_error(BSM_E_INVALID, err);
  if (!(err = load_tensor("B", B, tb)).empty()) return set_error(BSM_E_INVALID, err);
  if (c_order < 0 || c_order > kMaxModes || (c_order && !c_modes))
    return set_error(BSM_E_INVALID, "C: order must be 0..8 with its labels");
  std::vector<int32_t> cm(c_modes, c_modes + c_order);
  // labels: each of C's from exactly one operand; shared labels not in C are contracted
  std::vector<int> free_a, free_b, contr_a, contr_b, c_from_a;  // operand mode positions
  for (int p = 0; p < c_order; ++p) {
    for (int x = 0; x < p; ++x)
      if (cm[size_t(x)] == cm[size_t(p)]) return set_error(BSM_E_INVALID, "C: a label appears twice");
    const int pa = ta.pos(cm[size_t(p)]), pb = tb.pos(cm[size_t(p)]);
    if (pa >= 0 && pb >= 0)
      return set_error(BSM_E_UNSUPPORTED, "a label in A, B and C (a batch index) is not supported");
    if (pa < 0 && pb < 0) return set_error(BSM_E_INVALID, "C: a label in neither A nor B");
    if (pa >= 0) free_a.push_back(pa);
    else free_b.push_back(pb);
  }
  for (int m = 0; m < ta.order; ++m) {
    const int32_t l = ta.modes[size_t(m)];
    if (std::find(cm.begin(), cm.end(), l) != cm.end()) continue;
    const int pb = tb.pos(l);
    if (pb < 0) return set_error(BSM_E_UNSUPPORTED, "a label of A only, summed out, is not supported");
    if (ta.sizes[size_t(m)] != tb.sizes[size_t(pb)])
      return set_error(BSM_E_MISMATCH, "a contracted mode has different tilings in A and B");
    contr_a.push_back(m);
    contr_b.push_back(pb);
  }
  for (int m = 0; m < tb.order; ++m)
    if (std::find(cm.begin(), cm.end(), tb.modes[size_t(m)]) == cm.end() && ta.pos(tb.modes[size_t(m)]) < 0)
      return set_error(BSM_E_UNSUPPORTED, "a label of B only, summed out, is not supported");
  // C's order lists A's free modes before B's: the matrix C is C itself
  bool c_identity = true;
  for (int p = 0; p < c_order; ++p)
    if (p < int(free_a.size()) ? ta.pos(cm[size_t(p)]) < 0 : tb.pos(cm[size_t(p)]) < 0) c_identity = false;

  bsm_tc_plan* p = new (std::nothrow) bsm_tc_plan;
  if (!p) return set_error(BSM_E_NOMEM, "host allocation failed");
  try {
    // matricized block counts and sizes: tuples, mixed radix, last mode fastest
    auto tiling = [&](const Tensor& t, const std::vector<int>& pos, std::vector<int64_t>& out) -> bool {
      int64_t n = 1;
      for (int x : pos) n *= t.nb[size_t(x)];
      if (n > (int64_t(1) << 31)) return false;
      out.assign(size_t(n), 1);
      for (int64_t r = 0; r < n; ++r) {
        int64_t rem = r, size = 1;
        for (size_t y = pos.size(); y-- > 0;) {
          const int64_t nbm = t.nb[size_t(pos[y])];
          size *= t.sizes[size_t(pos[y])][size_t(rem % nbm)];
          rem /= nbm;
        }
        if (size > 65535) return false;
        out[size_t(r)] = size;
      }
      return true;
    };
    std::vector<int64_t> rs, ks, cs;
    if (!tiling(ta, free_a, rs) || !tiling(ta, contr_a, ks) || !tiling(tb, free_b, cs)) {
      tc_free(p);
      return set_error(BSM_E_UNSUPPORTED, "a matricized block exceeds 65535 rows or columns, or a "
                                          "matricized dimension exceeds 2^31 blocks");
    }
    const int64_t M = int64_t(rs.size()), K = int64_t(ks.size()), N = int64_t(cs.size());
    std::vector<uint64_t> abits(size_t(M * ((K + 63) / 64)), 0), bbits(size_t(K * ((N + 63) / 64)), 0);
    int64_t ta_elems = 0, tb_elems = 0;
    matricize(ta, free_a, contr_a, K, abits, p->a_mat, p->pa, ta_elems);
    matricize(tb, contr_b, free_b, N, bbits, p->b_mat, p->pb, tb_elems);
    // an operand already in matrix order is used in place
    std::vector<int> la(free_a), lb(contr_b);
    la.insert(la.end(), contr_a.begin(), contr_a.end());
    lb.insert(lb.end(), free_b.begin(), free_b.end());
    bool ida = true, idb = true;
    for (int m = 0; m < ta.order; ++m) ida = ida && la[size_t(m)] == m;
    for (int m = 0; m < tb.order; ++m) idb = idb && lb[size_t(m)] == m;
    if (ida) p->pa.clear();
    if (idb) p->pb.clear();
    p->c_f32 = o.out == BSM_OUT_F32;
    bsm_options om = o;
    if (!c_identity) om.out = BSM_OUT_F64;  // the matrix C is a workspace, C is written by the pass
    bsm_status st = bsm_plan_create(&p->mat, M, rs.data(), K, ks.data(), N, cs.data(),
                                    abits.data(), bbits.data(), &om);
    if (st != BSM_OK) {
      tc_free(p);
      return st;
    }
    bsm_plan_info im;
    bsm_plan_query(p->mat, &im);
    p->c_mat = im.c_elems;
    // C: matrix blocks (i, j) row-major -> C's tensor blocks, row-major over C's grid
    std::vector<uint64_t> mbits(size_t(M * ((N + 63) / 64)));
    bsm_plan_c_shape(p->mat, mbits.data());
    std::vector<int64_t> c_nb;  // C's block counts, mode after mode
    std::vector<const std::vector<int64_t>*> c_sz;
    for (int32_t l : cm) {
      const int x = ta.pos(l);
      const Tensor& t = x >= 0 ? ta : tb;
      const int y = x >= 0 ? x : tb.pos(l);
      c_nb.push_back(t.nb[size_t(y)]);
      c_sz.push_back(&t.sizes[size_t(y)]);
    }
    int64_t cgrid = 1;
    for (int64_t v : c_nb) cgrid *= v;
    p->c_bits.assign(size_t((cgrid + 63) / 64), 0);
    struct CB { int64_t flat, moff, n; int32_t ext[kMaxModes]; };  // ext in C's mode order
    std::vector<CB> cbs;
    const int64_t wn = (N + 63) / 64;
    int64_t moff = 0;
    const int na = int(free_a.size()), nbf = int(free_b.size());
    for (int64_t i = 0; i < M; ++i)
      for (int64_t j = 0; j < N; ++j) {
        if (!((mbits[size_t(i * wn + j / 64)] >> (j % 64)) & 1)) continue;
        // block indices of C's modes: free_a from i, free_b from j (C order within each)
        int64_t ia[kMaxModes], ib[kMaxModes];
        int64_t r = i;
        for (int x = na; x-- > 0;) { ia[x] = r % ta.nb[size_t(free_a[size_t(x)])]; r /= ta.nb[size_t(free_a[size_t(x)])]; }
        r = j;
        for (int x = nbf; x-- > 0;) { ib[x] = r % tb.nb[size_t(free_b[size_t(x)])]; r /= tb.nb[size_t(free_b[size_t(x)])]; }
        CB c{};
        int xa = 0, xb = 0;
        c.flat = 0;
        c.n = rs[size_t(i)] * cs[size_t(j)];
        for (int q = 0; q < c_order; ++q) {
          const int64_t bi = ta.pos(cm[size_t(q)]) >= 0 ? ia[xa++] : ib[xb++];
          c.flat = c.flat * c_nb[size_t(q)] + bi;
          c.ext[q] = int32_t((*c_sz[size_t(q)])[size_t(bi)]);
        }
        c.moff = moff;
        moff += c.n;
        p->c_bits[size_t(c.flat / 64)] |= uint64_t(1) << (c.flat % 64);
        cbs.push_back(c);
      }
    std::sort(cbs.begin(), cbs.end(), [](const CB& x, const CB& y) { return x.flat < y.flat; });
    int64_t toff = 0;
    if (!c_identity) {
      // source = the matrix block, modes in matrix order (A's free modes, then B's, each in C's
      // order); destination = the tensor block, row-major over C's modes
      std::vector<int> morder;  // C positions in matrix order
      for (int q = 0; q < c_order; ++q)
        if (ta.pos(cm[size_t(q)]) >= 0) morder.push_back(q);
      for (int q = 0; q < c_order; ++q)
        if (ta.pos(cm[size_t(q)]) < 0) morder.push_back(q);
      for (const CB& c : cbs) {
        PermBlock pbk{};
        pbk.src_off = c.moff;
        pbk.dst_off = toff;
        pbk.order = c_order;
        int64_t tstride[kMaxModes];
        int64_t s = 1;
        for (int q = c_order; q-- > 0;) { tstride[q] = s; s *= c.ext[q]; }
        for (int x = 0; x < c_order; ++x) {
          pbk.ext[x] = c.ext[morder[size_t(x)]];
          pbk.dst_stride[x] = tstride[morder[size_t(x)]];
        }
        p->pc.push_back(pbk);
        toff += c.n;
      }
    } else {
      toff = moff;
    }
    p->info.M = M;
    p->info.K = K;
    p->info.N = N;
    p->info.a_blocks = im.a_blocks;
    p->info.b_blocks = im.b_blocks;
    p->info.c_blocks = im.c_blocks;
    p->info.a_elems = ta_elems;
    p->info.b_elems = tb_elems;
    p->info.c_elems = toff;
    p->info.useful_flops = im.useful_flops;
    p->info.tasks = im.tasks;
    p->info.permute_a = p->pa.empty() ? 0 : 1;
    p->info.permute_b = p->pb.empty() ? 0 : 1;
    p->info.permute_c = c_identity ? 0 : 1;
    p->info.workspace_bytes = im.workspace_bytes +
                              (p->info.permute_a ? p->a_mat * 8 : 0) +
                              (p->info.permute_b ? p->b_mat * 8 : 0) +
                              (p->info.permute_c ? p->c_mat * 8 : 0);
    // the tables stay inside their buffers, and the matricized sizes agree with the plan's
    auto inside = [](const std::vector<PermBlock>& t, int64_t src_n, int64_t dst_n) {
      for (const PermBlock& b : t) {
        int64_t n = 1, last = 0;
        for (int m = 0; m < b.order; ++m) {
          n *= b.ext[m];
          last += int64_t(b.ext[m] - 1) * b.dst_stride[m];
        }
        if (n > 0 && (b.src_off < 0 || b.src_off + n > src_n || b.dst_off < 0 || b.dst_off + last >= dst_n))
          return false;
      }
      return true;
    };
    // pieces: A and B by kind; C element by element (it may accumulate or round to FP32)
    for (const PermBlock& b : p->pa) lower(b, false, p->xa);
    for (const PermBlock& b : p->pb) lower(b, false, p->xb);
    for (const PermBlock& b : p->pc) lower(b, true, p->xc);
    auto pieces_inside = [](const Pass& x, int64_t src_n, int64_t dst_n) {
      for (const CopyBlock& b : x.copy)
        if (b.src_off < 0 || b.dst_off < 0 || b.src_off + b.n > src_n || b.dst_off + b.n > dst_n)
          return false;
      for (const XposeBlock& b : x.xpose)
        if (b.src_off < 0 || b.dst_off < 0 ||
            b.src_off + int64_t(b.rows - 1) * b.ld_src + b.cols > src_n ||
            b.dst_off + int64_t(b.cols - 1) * b.ld_dst + b.rows > dst_n)
          return false;
      for (const PermBlock& b : x.perm) {
        int64_t last = 0;
        for (int m = 0; m < b.order; ++m) last += int64_t(b.ext[m] - 1) * b.dst_stride[m];
        if (b.e0 < 0 || b.e1 - b.e0 > kPermPiece || b.src_off + b.e1 > src_n ||
            b.dst_off + last >= dst_n || b.e1 > (int64_t(1) << 32))
          return false;
      }
      return true;
    };
    if (!pieces_inside(p->xa, ta_elems, p->a_mat) || !pieces_inside(p->xb, tb_elems, p->b_mat) ||
        !pieces_inside(p->xc, p->c_mat, p->info.c_elems)) {
      tc_free(p);
      return set_error(BSM_E_MISMATCH, "internal: a permutation piece leaves its buffers");
    }
    if (im.a_elems != p->a_mat || im.b_elems != p->b_mat || ta_elems != p->a_mat ||
        tb_elems != p->b_mat || toff != p->c_mat || !inside(p->pa, ta_elems, p->a_mat) ||
        !inside(p->pb, tb_elems, p->b_mat) || !inside(p->pc, p->c_mat, toff)) {
      tc_free(p);
      return set_error(BSM_E_MISMATCH, "internal: the matricized layouts disagree");
    }
  } catch (const std::bad_alloc&) {
    tc_free(p);
    return set_error(BSM_E_NOMEM, "host allocation failed while planning");
  }
  *out = p;
  return BSM_OK;
}

bsm_status bsm_tc_plan_query(const bsm_tc_plan* plan, bsm_tc_info* info) {
  if (!plan || !info) return set_error(BSM_E_INVALID, "null argument");
  *info = plan->info;
  return BSM_OK;
}

bsm_status bsm_tc_plan_c_shape(const bsm_tc_plan* plan, uint64_t* c_bits) {
  if (!plan || (!c_bits && !plan->c_bits.empty())) return set_error(BSM_E_INVALID, "null argument");
  if (!plan->c_bits.empty()) std::memcpy(c_bits, plan->c_bits.data(), plan->c_bits.size() * 8);
  return BSM_OK;
}

// Device tables and matricized buffers at the first execute.
static bsm_status tc_prepare(bsm_tc_plan* plan) {
  const bsm_tc_info& in = plan->info;
  bsm_status st;
  for (Pass* x : {&plan->xa, &plan->xb, &plan->xc})
    if ((st = upload_pass(*x)) != BSM_OK) return st;
  if (in.permute_a && plan->a_mat > 0)
    TC_HIP(hipMalloc(&plan->d_A, size_t(plan->a_mat) * 8), "hipMalloc(matricized A)");
  if (in.permute_b && plan->b_mat > 0)
    TC_HIP(hipMalloc(&plan->d_B, size_t(plan->b_mat) * 8), "hipMalloc(matricized B)");
  if (in.permute_c && plan->c_mat > 0)
    TC_HIP(hipMalloc(&plan->d_C, size_t(plan->c_mat) * 8), "hipMalloc(matricized C)");
  plan->ready = true;
  return BSM_OK;
}

bsm_status bsm_tc_execute(bsm_tc_plan* plan, double alpha, const double* dA, const double* dB,
                          void* dC, int accumulate, void* stream) {
  if (!plan) return set_error(BSM_E_INVALID, "plan is null");
  const bsm_tc_info& in = plan->info;
  if ((in.a_elems > 0 && !dA) || (in.b_elems > 0 && !dB) || (in.c_elems > 0 && !dC))
    return set_error(BSM_E_INVALID, "null tile buffer");
  if (accumulate != 0 && accumulate != 1) return set_error(BSM_E_INVALID, "accumulate must be 0 or 1");
  if (in.c_elems == 0) return BSM_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!plan->ready) {
    bsm_status st = tc_prepare(plan);
    if (st != BSM_OK) {
      // release what was allocated, so that a later call starts again from nothing
      std::vector<void**> slots = {reinterpret_cast<void**>(&plan->d_A),
                                   reinterpret_cast<void**>(&plan->d_B),
                                   reinterpret_cast<void**>(&plan->d_C)};
      for (Pass* x : {&plan->xa, &plan->xb, &plan->xc}) {
        slots.push_back(reinterpret_cast<void**>(&x->d_copy));
        slots.push_back(reinterpret_cast<void**>(&x->d_xpose));
        slots.push_back(reinterpret_cast<void**>(&x->d_perm));
      }
      for (void** sl : slots) {
        if (*sl) (void)hipFree(*sl);
        *sl = nullptr;
      }
      return st;
    }
  }
  const double* xa = dA;
  const double* xb = dB;
  bsm_status st;
  if (in.permute_a) {
    if ((st = run_pass(plan->xa, dA, plan->d_A, 0, 0, s, "matricize A")) != BSM_OK) return st;
    xa = plan->d_A;
  }
  if (in.permute_b) {
    if ((st = run_pass(plan->xb, dB, plan->d_B, 0, 0, s, "matricize B")) != BSM_OK) return st;
    xb = plan->d_B;
  }
  if (!in.permute_c) return bsm_execute(plan->mat, alpha, xa, xb, dC, accumulate, stream);
  st = bsm_execute(plan->mat, alpha, xa, xb, plan->d_C, 0, stream);
  if (st != BSM_OK) return st;
  return run_pass(plan->xc, plan->d_C, dC, plan->c_f32, accumulate, s, "C into its mode order");
}

bsm_status bsm_tc_plan_verify(bsm_tc_plan* plan, void* stream) {
  if (!plan) return set_error(BSM_E_INVALID, "plan is null");
  return bsm_plan_verify(plan->mat, stream);
}

bsm_status bsm_tc_plan_destroy(bsm_tc_plan* plan) {
  if (plan) tc_free(plan);
  return BSM_OK;
}

}  // extern "C"
