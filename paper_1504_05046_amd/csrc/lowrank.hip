// Block-rank-sparse left operand (Sec. 1 names block-rank sparsity, blocks of low rank, as the
// data sparsity the task formulation is a step towards): a present block of A is either dense or
// stored as factors A_ik = U V^T.  The product runs as two ordinary block-sparse products on the
// library's own kernels, so every factored block costs O(rho) instead of O(s_k) per output element:
//
//   stage 1   W_(ik)j = V_ik^T B_kj   for every factored (i,k) and present B_kj: a block-sparse
//             product with one row block per inner block k that has factored blocks, holding the
//             V^T of all of them stacked (sum of their ranks rows; one present block per row, at
//             inner block k), so that its C blocks are tall enough for full tiles;
//   stage 2   C = alpha [A_dense | U] [B ; W] (+ C): one product over the inner dimension extended
//             by one block per factored block (inner size rho_q), whose left operand holds the
//             dense blocks and the U factors and whose right operand is B with W's rows appended.
//
// Stage 2's C-shape is the C-shape of A B (row q of W has B's row k shape), so C keeps the
// ordinary layout.  Staging on the stream: the dense blocks and U factors are gathered into the
// stage-2 left operand, the V factors transposed into the stage-1 left operand, B copied in front
// of W, and each W_(ik)j (a run of whole rows of stage 1's stacked C block) copied to its place
// in stage 2's right operand.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/bsm.h"
#include "errors.hpp"
#include "kernels.hpp"
#include "staging.hpp"

using namespace bsm;

#define LR_HIP(call, what)                                                                  \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return set_error(BSM_E_HIP, std::string(what) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct bsm_lr_plan {
  bsm_plan* stage1 = nullptr;  // W = V^T B (absent when no block is factored)
  bsm_plan* main = nullptr;    // C = alpha [A_dense | U] [B ; W] (+ C)
  bsm_lr_info info{};
  int64_t a2_elems = 0, v_elems = 0, w_elems = 0;
  std::vector<CopyBlock> gather;  // caller's dense blocks and U factors -> stage-2 left operand
  std::vector<XposeBlock> vt;     // caller's V factors (s_k x rho) -> V^T blocks of stage 1
  std::vector<CopyBlock> restack; // stage 1's stacked W rows -> W_(ik)j blocks of stage 2
  CopyBlock* d_gather = nullptr;
  XposeBlock* d_vt = nullptr;
  CopyBlock* d_restack = nullptr;
  double* d_W = nullptr;          // stage 1's C (stacked W)
  double* d_A2 = nullptr;         // stage-2 left operand
  double* d_V1 = nullptr;         // stage-1 left operand
  double* d_B2 = nullptr;         // B followed by W
  bool ready = false;
};

static int64_t words_of(int64_t n) { return (n + 63) / 64; }
static bool bit_of(const uint64_t* bits, int64_t ncols, int64_t i, int64_t j) {
  return (bits[i * words_of(ncols) + j / 64] >> (j % 64)) & 1;
}

static bsm_status lr_prepare_buffers(bsm_lr_plan* p);

// Device buffers at the first execute; a failure part-way releases what was allocated.
static bsm_status lr_prepare(bsm_lr_plan* p) {
  if (p->ready) return BSM_OK;
  const bsm_status st = lr_prepare_buffers(p);
  if (st != BSM_OK) {
    void** slots[] = {reinterpret_cast<void**>(&p->d_gather), reinterpret_cast<void**>(&p->d_vt),
                      reinterpret_cast<void**>(&p->d_restack), reinterpret_cast<void**>(&p->d_W),
                      reinterpret_cast<void**>(&p->d_A2), reinterpret_cast<void**>(&p->d_V1),
                      reinterpret_cast<void**>(&p->d_B2)};
    for (void** s : slots) {
      if (*s) (void)hipFree(*s);
      *s = nullptr;
    }
  }
  return st;
}

static bsm_status lr_prepare_buffers(bsm_lr_plan* p) {
  auto up = [&](auto** dst, const auto& v) -> bsm_status {
    const size_t bytes = v.size() * sizeof(v[0]);
    if (!bytes) return BSM_OK;
    LR_HIP(hipMalloc(dst, bytes), "hipMalloc(low-rank tables)");
    LR_HIP(hipMemcpy(*dst, v.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy(low-rank tables)");
    return BSM_OK;
  };
  bsm_status st;
  if ((st = up(&p->d_gather, p->gather)) != BSM_OK) return st;
  if ((st = up(&p->d_vt, p->vt)) != BSM_OK) return st;
  if ((st = up(&p->d_restack, p->restack)) != BSM_OK) return st;
  if (p->w_elems > 0) LR_HIP(hipMalloc(&p->d_W, size_t(p->w_elems) * 8), "hipMalloc(stage-1 C)");
  if (p->a2_elems > 0) LR_HIP(hipMalloc(&p->d_A2, size_t(p->a2_elems) * 8), "hipMalloc(stage-2 A)");
  if (p->v_elems > 0) LR_HIP(hipMalloc(&p->d_V1, size_t(p->v_elems) * 8), "hipMalloc(stage-1 A)");
  const int64_t nb2 = p->info.b_elems + p->w_elems;
  if (nb2 > 0) LR_HIP(hipMalloc(&p->d_B2, size_t(nb2) * 8), "hipMalloc(B and W)");
  p->ready = true;
  return BSM_OK;
}

// Every run of a staging table inside its source and destination buffers (checked on the host
// before anything is launched).
static bool runs_inside(const std::vector<CopyBlock>& t, int64_t src_n, int64_t dst_n) {
  for (const CopyBlock& b : t)
    if (b.src_off < 0 || b.dst_off < 0 || b.n < 0 || b.src_off + b.n > src_n || b.dst_off + b.n > dst_n)
      return false;
  return true;
}
static bool blocks_inside(const std::vector<XposeBlock>& t, int64_t src_n, int64_t dst_n) {
  for (const XposeBlock& b : t) {
    if (b.rows <= 0 || b.cols <= 0) continue;
    const int64_t last_src = b.src_off + int64_t(b.rows - 1) * b.ld_src + b.cols - 1;
    const int64_t last_dst = b.dst_off + int64_t(b.cols - 1) * b.ld_dst + b.rows - 1;
    if (b.src_off < 0 || b.dst_off < 0 || last_src >= src_n || last_dst >= dst_n) return false;
  }
  return true;
}

static void lr_free(bsm_lr_plan* p) {
  if (p->stage1) bsm_plan_destroy(p->stage1);
  if (p->main) bsm_plan_destroy(p->main);
  // also the buffers of a preparation that failed part-way
  const std::initializer_list<void*> bufs = {
      static_cast<void*>(p->d_gather), static_cast<void*>(p->d_vt), static_cast<void*>(p->d_restack),
      static_cast<void*>(p->d_W), static_cast<void*>(p->d_A2), static_cast<void*>(p->d_V1),
      static_cast<void*>(p->d_B2)};
  bool any = false;
  for (void* ptr : bufs) any = any || ptr;
  if (any) {
    (void)hipDeviceSynchronize();
    for (void* ptr : bufs)
      if (ptr) (void)hipFree(ptr);
  }
  delete p;
}

extern "C" {

bsm_status bsm_lr_plan_create(bsm_lr_plan** out, int64_t M, const int64_t* row_sizes, int64_t K,
                              const int64_t* inner_sizes, int64_t N, const int64_t* col_sizes,
                              const uint64_t* a_bits, const int32_t* a_ranks,
                              const uint64_t* b_bits, const bsm_options* opt) {
  if (!out) return set_error(BSM_E_INVALID, "out is null");
  *out = nullptr;
  bsm_options o;
  bsm_options_default(&o);
  if (opt) o = *opt;
  if (o.elem != BSM_REAL) return set_error(BSM_E_UNSUPPORTED, "block-rank-sparse plans are real");
  if (o.trans_a || o.trans_b)
    return set_error(BSM_E_UNSUPPORTED, "block-rank-sparse plans take untransposed operands");
  if (M < 0 || K < 0 || N < 0) return set_error(BSM_E_INVALID, "negative block count");
  if ((M && !row_sizes) || (K && !inner_sizes) || (N && !col_sizes))
    return set_error(BSM_E_INVALID, "null size vector");
  for (int64_t x = 0; x < M; ++x)
    if (row_sizes[x] < 1 || row_sizes[x] > 65535) return set_error(BSM_E_INVALID, "row_sizes out of range");
  for (int64_t x = 0; x < K; ++x)
    if (inner_sizes[x] < 1 || inner_sizes[x] > 65535)
      return set_error(BSM_E_INVALID, "inner_sizes out of range");
  const int64_t wk = words_of(K), wn = words_of(N);
  if ((M * wk && !a_bits) || (K * wn && !b_bits)) return set_error(BSM_E_INVALID, "null bitmap");
  if (K % 64)
    for (int64_t i = 0; i < M; ++i)
      if (a_bits[i * wk + wk - 1] & (~uint64_t(0) << (K % 64)))
        return set_error(BSM_E_INVALID, "a_bits: padding bit set in row " + std::to_string(i));
  bsm_lr_plan* p = new (std::nothrow) bsm_lr_plan;
  if (!p) return set_error(BSM_E_NOMEM, "host allocation failed");
  try {
    // walk A's present blocks in packed order: caller's offsets, ranks, factored blocks
    struct Fac { int64_t i, k, rho, u_off, v_off; };
    std::vector<Fac> fac;
    std::vector<int64_t> dense_off(size_t(M * K), -1);
    int64_t pos = 0, q = 0, nblocks = 0;
    for (int64_t i = 0; i < M; ++i)
      for (int64_t k = 0; k < K; ++k) {
        if (!bit_of(a_bits, K, i, k)) continue;
        ++nblocks;
        const int32_t rho = a_ranks ? a_ranks[q] : 0;
        ++q;
        if (rho < 0 || rho > 65535) {
          lr_free(p);
          return set_error(BSM_E_INVALID, "a_ranks: rank out of range [0, 65535]");
        }
        if (rho == 0) {
          dense_off[size_t(i * K + k)] = pos;
          pos += row_sizes[i] * inner_sizes[k];
        } else {
          fac.push_back(Fac{i, k, rho, pos, pos + row_sizes[i] * rho});
          pos += (row_sizes[i] + inner_sizes[k]) * rho;
        }
      }
    if (nblocks > 0 && !a_ranks) {
      lr_free(p);
      return set_error(BSM_E_INVALID, "a_ranks is null");
    }
    const int64_t Q = int64_t(fac.size());
    // stage 2: inner dimension K + Q; A2 row i = dense bits, then the factored blocks of row i
    const int64_t K2 = K + Q, wk2 = words_of(K2);
    std::vector<int64_t> inner2(inner_sizes, inner_sizes + K);
    for (const Fac& f : fac) inner2.push_back(f.rho);
    std::vector<uint64_t> a2(size_t(M * wk2), 0), b2(size_t(K2 * wn), 0);
    for (int64_t i = 0; i < M; ++i)
      for (int64_t k = 0; k < K; ++k)
        if (dense_off[size_t(i * K + k)] >= 0) a2[size_t(i * wk2 + k / 64)] |= uint64_t(1) << (k % 64);
    for (int64_t f = 0; f < Q; ++f) {
      const int64_t kk = K + f;
      a2[size_t(fac[size_t(f)].i * wk2 + kk / 64)] |= uint64_t(1) << (kk % 64);
    }
    if (K * wn) std::memcpy(b2.data(), b_bits, size_t(K * wn) * 8);
    for (int64_t f = 0; f < Q; ++f)
      std::memcpy(b2.data() + (K + f) * wn, b_bits + fac[size_t(f)].k * wn, size_t(wn) * 8);
    // gather table: A2 packed in row-major block order over (i, k'), k' < K dense, then factors
    int64_t a2pos = 0;
    size_t fq = 0;
    for (int64_t i = 0; i < M; ++i) {
      for (int64_t k = 0; k < K; ++k) {
        const int64_t o = dense_off[size_t(i * K + k)];
        if (o < 0) continue;
        const int64_t n = row_sizes[i] * inner_sizes[k];
        push_copy(p->gather, o, a2pos, n);
        a2pos += n;
      }
      for (; fq < fac.size() && fac[fq].i == i; ++fq) {
        const int64_t n = row_sizes[i] * fac[fq].rho;
        push_copy(p->gather, fac[fq].u_off, a2pos, n);
        a2pos += n;
      }
    }
    p->a2_elems = a2pos;
    // stage 1: one row block g per inner block k with factored blocks, R_g = the sum of their
    // ranks rows; factored block q sits at rows [o_q, o_q + rho_q) of its group (groups in k
    // order, blocks in row order inside a group).  Row block g has one block, at inner block k:
    // the stacked V^T (R_g x s_k), each V^T written by transposing the caller's s_k x rho V.
    std::vector<int64_t> group_of_k(size_t(K), -1), rows1, first_row(size_t(Q), 0), gk;
    std::vector<std::vector<int64_t>> members;
    constexpr int64_t kUsed = -2;  // inner block with factored blocks, numbered in k order below
    for (int64_t f = 0; f < Q; ++f) group_of_k[size_t(fac[size_t(f)].k)] = kUsed;
    for (int64_t k = 0; k < K; ++k)
      if (group_of_k[size_t(k)] == kUsed) {
        group_of_k[size_t(k)] = int64_t(gk.size());
        gk.push_back(k);
        rows1.push_back(0);
        members.emplace_back();
      }
    for (int64_t f = 0; f < Q; ++f) {
      const int64_t g = group_of_k[size_t(fac[size_t(f)].k)];
      first_row[size_t(f)] = rows1[size_t(g)];
      rows1[size_t(g)] += fac[size_t(f)].rho;
      members[size_t(g)].push_back(f);
    }
    const int64_t G = int64_t(gk.size());
    for (int64_t g = 0; g < G; ++g)
      if (rows1[size_t(g)] > 65535) {
        lr_free(p);
        return set_error(BSM_E_UNSUPPORTED, "the ranks of the factored blocks of one inner block "
                                            "sum to more than 65535");
      }
    std::vector<uint64_t> a1(size_t(G * wk), 0);
    std::vector<int64_t> a1_off(size_t(G), 0);
    int64_t v1pos = 0;
    for (int64_t g = 0; g < G; ++g) {
      const int64_t k = gk[size_t(g)];
      a1[size_t(g * wk + k / 64)] |= uint64_t(1) << (k % 64);
      a1_off[size_t(g)] = v1pos;
      v1pos += rows1[size_t(g)] * inner_sizes[k];
    }
    for (int64_t f = 0; f < Q; ++f) {
      const Fac& x = fac[size_t(f)];
      const int64_t g = group_of_k[size_t(x.k)];
      push_transpose(p->vt, x.v_off, a1_off[size_t(g)] + first_row[size_t(f)] * inner_sizes[x.k],
                     int32_t(inner_sizes[x.k]), int32_t(x.rho));
    }
    p->v_elems = v1pos;
    // stage 1's C: block (g, j) at the packed offset of the stacked R_g x t_j blocks; W_(q)j is
    // rows [o_q, o_q + rho_q) of it.  Stage 2's right operand: B's blocks, then W's blocks in
    // row-major order over (K + q, j).
    {
      std::vector<int64_t> c1_off(size_t(G * N), -1);
      int64_t c1 = 0;
      for (int64_t g = 0; g < G; ++g)
        for (int64_t j = 0; j < N; ++j)
          if (bit_of(b_bits, N, gk[size_t(g)], j)) {
            c1_off[size_t(g * N + j)] = c1;
            c1 += rows1[size_t(g)] * col_sizes[j];
          }
      p->w_elems = c1;
      int64_t bpos = 0;  // offsets relative to the start of W in stage 2's right operand
      for (int64_t f = 0; f < Q; ++f) {
        const Fac& x = fac[size_t(f)];
        const int64_t g = group_of_k[size_t(x.k)];
        for (int64_t j = 0; j < N; ++j) {
          if (!bit_of(b_bits, N, x.k, j)) continue;
          const int64_t n = x.rho * col_sizes[j];
          push_copy(p->restack, c1_off[size_t(g * N + j)] + first_row[size_t(f)] * col_sizes[j],
                    bpos, n);
          bpos += n;
        }
      }
    }
    bsm_options o1 = o;
    o1.out = BSM_OUT_F64;
    o1.k_window = 0;
    o1.record_timings = 0;
    o1.tile = 0;
    o1.tune_cache = nullptr;
    bsm_status st;
    if (Q > 0) {
      st = bsm_plan_create(&p->stage1, G, rows1.data(), K, inner_sizes, N, col_sizes, a1.data(),
                           b_bits, &o1);
      if (st != BSM_OK) {
        lr_free(p);
        return st;
      }
      bsm_plan_info i1;
      bsm_plan_query(p->stage1, &i1);
      if (i1.c_elems != p->w_elems) {
        lr_free(p);
        return set_error(BSM_E_MISMATCH, "internal: stage-1 C layout differs from its restack table");
      }
      p->info.useful_flops += i1.useful_flops;
      p->info.tasks += i1.tasks;
      p->info.workspace_bytes += i1.workspace_bytes;
    }
    st = bsm_plan_create(&p->main, M, row_sizes, K2, inner2.data(), N, col_sizes, a2.data(),
                         b2.data(), &o);
    if (st != BSM_OK) {
      lr_free(p);
      return st;
    }
    bsm_plan_info im;
    bsm_plan_query(p->main, &im);
    p->info.M = M;
    p->info.K = K;
    p->info.N = N;
    p->info.a_blocks = nblocks;
    p->info.factored_blocks = Q;
    p->info.a_elems = pos;
    p->info.b_elems = 0;
    for (int64_t k = 0; k < K; ++k)
      for (int64_t j = 0; j < N; ++j)
        if (bit_of(b_bits, N, k, j)) p->info.b_elems += inner_sizes[k] * col_sizes[j];
    if (!runs_inside(p->gather, pos, p->a2_elems) || !blocks_inside(p->vt, pos, p->v_elems) ||
        !runs_inside(p->restack, p->w_elems, p->w_elems) || im.a_elems != p->a2_elems ||
        im.b_elems != p->info.b_elems + p->w_elems) {
      lr_free(p);
      return set_error(BSM_E_MISMATCH, "internal: a staging table leaves its buffers");
    }
    p->info.c_blocks = im.c_blocks;
    p->info.c_elems = im.c_elems;
    p->info.useful_flops += im.useful_flops;
    p->info.tasks += im.tasks;
    // the same product with every block of A dense: 2 r_i s_k t_j over (i,k,j) triples
    std::vector<double> brow(size_t(K), 0.0);
    for (int64_t k = 0; k < K; ++k)
      for (int64_t j = 0; j < N; ++j)
        if (bit_of(b_bits, N, k, j)) brow[size_t(k)] += double(col_sizes[j]);
    for (int64_t i = 0; i < M; ++i)
      for (int64_t k = 0; k < K; ++k)
        if (bit_of(a_bits, K, i, k))
          p->info.dense_flops += 2.0 * double(row_sizes[i]) * double(inner_sizes[k]) * brow[size_t(k)];
    p->info.workspace_bytes += im.workspace_bytes + (p->a2_elems + p->v_elems + p->info.b_elems +
                                                     2 * p->w_elems) * 8 +
                               int64_t((p->gather.size() + p->restack.size()) * sizeof(CopyBlock) +
                                       p->vt.size() * sizeof(XposeBlock));
  } catch (const std::bad_alloc&) {
    lr_free(p);
    return set_error(BSM_E_NOMEM, "host allocation failed while planning");
  }
  *out = p;
  return BSM_OK;
}

bsm_status bsm_lr_plan_query(const bsm_lr_plan* plan, bsm_lr_info* info) {
  if (!plan || !info) return set_error(BSM_E_INVALID, "null argument");
  *info = plan->info;
  return BSM_OK;
}

bsm_status bsm_lr_plan_c_offsets(const bsm_lr_plan* plan, int64_t* c_offsets) {
  if (!plan) return set_error(BSM_E_INVALID, "plan is null");
  return bsm_plan_c_offsets(plan->main, c_offsets);
}

bsm_status bsm_lr_execute(bsm_lr_plan* plan, double alpha, const double* dA, const double* dB,
                          void* dC, int accumulate, void* stream) {
  if (!plan) return set_error(BSM_E_INVALID, "plan is null");
  const bsm_lr_info& in = plan->info;
  if ((in.a_elems > 0 && !dA) || (in.b_elems > 0 && !dB) || (in.c_elems > 0 && !dC))
    return set_error(BSM_E_INVALID, "null tile buffer");
  if (accumulate != 0 && accumulate != 1) return set_error(BSM_E_INVALID, "accumulate must be 0 or 1");
  bsm_plan_info im;
  bsm_plan_query(plan->main, &im);
  const uintptr_t c0 = uintptr_t(dC), c1 = c0 + uintptr_t(in.c_elems * (im.out == BSM_OUT_F32 ? 4 : 8));
  for (auto [ptr, n] : {std::pair<const double*, int64_t>{dA, in.a_elems}, {dB, in.b_elems}})
    if (n > 0 && in.c_elems > 0 && uintptr_t(ptr) < c1 && c0 < uintptr_t(ptr + n))
      return set_error(BSM_E_INVALID, "C overlaps A or B");
  if (in.c_elems == 0) return BSM_OK;
  bsm_status st = lr_prepare(plan);
  if (st != BSM_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  LR_HIP(launch_copy_blocks(plan->d_gather, int64_t(plan->gather.size()), dA, plan->d_A2, s),
         "gather dense blocks and U factors");
  LR_HIP(launch_transpose_f64(plan->d_vt, int64_t(plan->vt.size()), dA, plan->d_V1, s),
         "transpose V factors");
  if (in.b_elems > 0)
    LR_HIP(hipMemcpyAsync(plan->d_B2, dB, size_t(in.b_elems) * 8, hipMemcpyDeviceToDevice, s),
           "copy B");
  if (plan->stage1 && plan->w_elems > 0) {
    st = bsm_execute(plan->stage1, 1.0, plan->d_V1, dB, plan->d_W, 0, stream);
    if (st != BSM_OK) return st;
    LR_HIP(launch_copy_blocks(plan->d_restack, int64_t(plan->restack.size()), plan->d_W,
                              plan->d_B2 + in.b_elems, s), "place W blocks");
  }
  return bsm_execute(plan->main, alpha, plan->d_A2, plan->d_B2, dC, accumulate, stream);
}

bsm_status bsm_lr_plan_verify(bsm_lr_plan* plan, void* stream) {
  if (!plan) return set_error(BSM_E_INVALID, "plan is null");
  if (plan->stage1) {
    bsm_status st = bsm_plan_verify(plan->stage1, stream);
    if (st != BSM_OK) return st;
  }
  return bsm_plan_verify(plan->main, stream);
}

bsm_status bsm_lr_plan_destroy(bsm_lr_plan* plan) {
  if (plan) lr_free(plan);
  return BSM_OK;
}

}  // extern "C"
