/*
 * Plain CPU reference for the block-sparse product -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may load this library.
 * It shares no code with the GPU library: no headers, helpers or tables in common.
 *
 * What it computes (paper Sec. 2.1, the rank-k update C_ij <- A_ik B_kj + C_ij summed over k, and
 * Alg. 1's local update C <- alpha A(*,k) B(k,*) + C; Sec. 3.2 splits each update into a product
 * C^(k)_ij = A_ik B_kj and a reduction C_ij += C^(k)_ij, which changes only when the terms are
 * added, not which terms are added):
 *
 *   tilings r[0..M), s[0..K), t[0..N) (block sizes of any value, Sec. 3.2);
 *   block-shape masks Ahat (M x K) and Bhat (K x N);
 *   C-shape   Chat_ij = OR_k (Ahat_ik AND Bhat_kj);
 *   values    C_ij = alpha * sum_{k : Ahat_ik and Bhat_kj} A_ik B_kj  (+ C_ij when accumulating),
 *             for every (i,j) with Chat_ij; absent blocks are zero and are not stored.
 *
 * Storage (the library's input format): bit (i,j) of a shape is bit j%64 of word
 * i*ceil(ncols/64) + j/64; present blocks are packed in row-major block order, each block
 * row-major with leading dimension equal to its column count.
 *
 * Arithmetic: FP64, built without contraction (-ffp-contract=off, no fast-math), plain loops in
 * i-k-j order, k blocks ascending, one OpenMP thread per whole C block, so the result does not
 * depend on the thread count.  An optional long-double accumulator gives a tighter reference.
 *
 * Transposed operands (the SUMMA variants of Sec. 2.1 that multiply by a transpose):
 * C = alpha op(A) op(B) (+ C), op(X) = X or X^T.  The tilings always describe the product
 * (r: rows of C and of op(A), s: the inner dimension, t: columns of C and of op(B)).  A transposed
 * operand is stored as the transposed block matrix: for op(A) = A^T the stored matrix has K x M
 * blocks, its shape bit (k, i) and its block (k, i) of s_k x r_i elements, row-major, packed in
 * the stored matrix's row-major block order; likewise op(B) = B^T is stored as N x K blocks of
 * t_j x s_k elements.  op(A)_ik is then the transpose of the stored block (k, i).
 *
 * Complex elements (Sec. 4.3 names real and complex element types as both supported): the same
 * product over complex blocks, each element stored as two doubles (real part, then imaginary
 * part), offsets counted in complex elements.  Here op(X) may also be the adjoint X^H (transpose
 * and conjugate), and alpha is complex.  Every complex multiply-add is written out in real
 * arithmetic: (ar + i ai)(br + i bi) = (ar br - ai bi) + i (ar bi + ai br).
 *
 * Block-rank-sparse operands (Sec. 1 names block-rank sparsity, data-sparse blocks of low rank,
 * as the structure the task formulation targets): a present block of A may be stored as factors,
 * A_ik = U V^T with U r_i x rho and V s_k x rho (both row-major, U first); rho = 0 marks a dense
 * block.  The packed buffer holds each present block in row-major block order, r_i s_k elements
 * for a dense block and (r_i + s_k) rho for a factored one.  The oracle multiplies out every
 * factored block (plain loops, FP64) and then takes the ordinary product.
 *
 * Also here: the paper's two closed forms, the concurrent-iteration limit (Eq. 1) and the
 * per-node memory overhead of one SUMMA iteration (Eq. 2).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int64_t words_of(int64_t ncols) { return (ncols + 63) / 64; }

static int bit_at(const uint64_t* bits, int64_t ncols, int64_t i, int64_t j) {
  return (int)((bits[i * words_of(ncols) + j / 64] >> (j % 64)) & 1u);
}

int64_t oracle_words(int64_t ncols) { return words_of(ncols); }

/* Threads the OpenMP loops below use. */
int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Sets the threads of the OpenMP loops below (n >= 1) for later calls from the calling thread;
 * returns the previous count.  Timing only: the results do not depend on it. */
int oracle_set_threads(int n) {
  const int prev = oracle_threads();
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
  return prev;
}

/* Chat = boolean product of the two shapes, by the definition: a triple loop over (i, j, k). */
int oracle_shape_product(int64_t M, int64_t K, int64_t N, const uint64_t* a_bits,
                         const uint64_t* b_bits, uint64_t* c_bits) {
  int64_t wn = words_of(N);
  memset(c_bits, 0, (size_t)(M * wn) * sizeof(uint64_t));
  for (int64_t i = 0; i < M; ++i)
    for (int64_t j = 0; j < N; ++j) {
      int present = 0;
      for (int64_t k = 0; k < K && !present; ++k)
        present = bit_at(a_bits, K, i, k) && bit_at(b_bits, N, k, j);
      if (present) c_bits[i * wn + j / 64] |= (uint64_t)1 << (j % 64);
    }
  return 0;
}

/* Offsets (in elements) of the present blocks of an R x C block matrix in the packed layout;
 * off[i*C + j] = -1 for an absent block.  Returns the total number of stored elements. */
int64_t oracle_block_offsets(int64_t R, int64_t C, const int64_t* rsz, const int64_t* csz,
                             const uint64_t* bits, int64_t* off) {
  int64_t pos = 0;
  for (int64_t i = 0; i < R; ++i)
    for (int64_t j = 0; j < C; ++j) {
      if (bit_at(bits, C, i, j)) {
        off[i * C + j] = pos;
        pos += rsz[i] * csz[j];
      } else {
        off[i * C + j] = -1;
      }
    }
  return pos;
}

/* Useful flops: 2 r_i s_k t_j summed over every triple with both blocks present. */
double oracle_useful_flops(int64_t M, int64_t K, int64_t N, const int64_t* r, const int64_t* s,
                           const int64_t* t, const uint64_t* a_bits, const uint64_t* b_bits) {
  double f = 0.0;
  for (int64_t i = 0; i < M; ++i)
    for (int64_t k = 0; k < K; ++k) {
      if (!bit_at(a_bits, K, i, k)) continue;
      for (int64_t j = 0; j < N; ++j)
        if (bit_at(b_bits, N, k, j)) f += 2.0 * (double)r[i] * (double)s[k] * (double)t[j];
    }
  return f;
}

typedef struct {
  int64_t M, K, N;
  const int64_t *r, *s, *t;
  const uint64_t *a_bits, *b_bits; /* as stored (transposed shapes when ta / tb) */
  int ta, tb;                      /* op(A) = A^T, op(B) = B^T */
  int64_t *a_off, *b_off; /* stored packed offsets: M*K (or K*M) and K*N (or N*K), -1 = absent */
} problem;

static int setup(problem* p, int64_t M, int64_t K, int64_t N, const int64_t* r, const int64_t* s,
                 const int64_t* t, const uint64_t* a_bits, const uint64_t* b_bits, int ta, int tb) {
  p->M = M; p->K = K; p->N = N; p->r = r; p->s = s; p->t = t;
  p->a_bits = a_bits; p->b_bits = b_bits;
  p->ta = ta; p->tb = tb;
  p->a_off = (int64_t*)malloc((size_t)(M * K > 0 ? M * K : 1) * sizeof(int64_t));
  p->b_off = (int64_t*)malloc((size_t)(K * N > 0 ? K * N : 1) * sizeof(int64_t));
  if (!p->a_off || !p->b_off) return -1;
  if (ta) oracle_block_offsets(K, M, s, r, a_bits, p->a_off);
  else oracle_block_offsets(M, K, r, s, a_bits, p->a_off);
  if (tb) oracle_block_offsets(N, K, t, s, b_bits, p->b_off);
  else oracle_block_offsets(K, N, s, t, b_bits, p->b_off);
  return 0;
}

/* stored offset of op(A)_ik and op(B)_kj (-1 when absent) */
static int64_t a_at(const problem* p, int64_t i, int64_t k) {
  return p->ta ? p->a_off[k * p->M + i] : p->a_off[i * p->K + k];
}
static int64_t b_at(const problem* p, int64_t k, int64_t j) {
  return p->tb ? p->b_off[j * p->K + k] : p->b_off[k * p->N + j];
}

/* The C-shape of op(A) op(B), from the stored shapes. */
static void shape_of_product(const problem* p, uint64_t* c_bits) {
  int64_t wn = words_of(p->N);
  memset(c_bits, 0, (size_t)(p->M * wn) * sizeof(uint64_t));
  for (int64_t i = 0; i < p->M; ++i)
    for (int64_t j = 0; j < p->N; ++j)
      for (int64_t k = 0; k < p->K; ++k)
        if (a_at(p, i, k) >= 0 && b_at(p, k, j) >= 0) {
          c_bits[i * wn + j / 64] |= (uint64_t)1 << (j % 64);
          break;
        }
}

static void teardown(problem* p) { free(p->a_off); free(p->b_off); }

/* One C block: out (r_i x t_j, row-major) = sum over present k of A_ik B_kj, k ascending,
 * elements in i-k-j order. Returns 1 if the block is present in Chat. */
static int block_product(const problem* p, const double* A, const double* B, int64_t i, int64_t j,
                         double* out, int extended) {
  int64_t h = p->r[i], w = p->t[j];
  int present = 0;
  long double* acc = NULL;
  if (extended) acc = (long double*)calloc((size_t)(h * w > 0 ? h * w : 1), sizeof(long double));
  for (int64_t e = 0; e < h * w; ++e) out[e] = 0.0;
  for (int64_t k = 0; k < p->K; ++k) {
    int64_t ao = a_at(p, i, k), bo = b_at(p, k, j);
    if (ao < 0 || bo < 0) continue;
    present = 1;
    int64_t d = p->s[k];
    const double* a = A + ao; /* op(A)_ik: h x d; stored d x h when transposed */
    const double* b = B + bo; /* op(B)_kj: d x w; stored w x d when transposed */
    for (int64_t x = 0; x < h; ++x)
      for (int64_t y = 0; y < d; ++y) {
        double av = p->ta ? a[y * h + x] : a[x * d + y];
        for (int64_t z = 0; z < w; ++z) {
          double bv = p->tb ? b[z * d + y] : b[y * w + z];
          if (extended) acc[x * w + z] += (long double)av * (long double)bv;
          else out[x * w + z] += av * bv;
        }
      }
  }
  if (extended) {
    for (int64_t e = 0; e < h * w; ++e) out[e] = (double)acc[e];
    free(acc);
  }
  return present;
}

/* Full product.  C is the packed C buffer (layout from the C-shape); with accumulate = 0 it is
 * overwritten, with accumulate = 1 it must hold the previous C and receives alpha*AB + C. */
int oracle_bsmm(int64_t M, int64_t K, int64_t N, const int64_t* r, const int64_t* s,
                const int64_t* t, const uint64_t* a_bits, const uint64_t* b_bits, const double* A,
                const double* B, double alpha, int accumulate, double* C, int extended, int ta,
                int tb) {
  problem p;
  if (setup(&p, M, K, N, r, s, t, a_bits, b_bits, ta, tb)) { teardown(&p); return -1; }
  int64_t wn = words_of(N);
  uint64_t* c_bits = (uint64_t*)calloc((size_t)(M * wn > 0 ? M * wn : 1), sizeof(uint64_t));
  int64_t* c_off = (int64_t*)malloc((size_t)(M * N > 0 ? M * N : 1) * sizeof(int64_t));
  if (!c_bits || !c_off) { free(c_bits); free(c_off); teardown(&p); return -1; }
  shape_of_product(&p, c_bits);
  oracle_block_offsets(M, N, r, t, c_bits, c_off);
  int status = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < M * N; ++q) {
    int64_t i = q / N, j = q % N;
    int64_t co = c_off[q];
    if (co < 0) continue;
    int64_t hw = r[i] * t[j];
    double* tmp = (double*)malloc((size_t)(hw > 0 ? hw : 1) * sizeof(double));
    if (!tmp) { status = -1; continue; }
    block_product(&p, A, B, i, j, tmp, extended);
    for (int64_t e = 0; e < hw; ++e) {
      double v = alpha * tmp[e];
      C[co + e] = accumulate ? v + C[co + e] : v;
    }
    free(tmp);
  }
  free(c_bits); free(c_off); teardown(&p);
  return status;
}

/* Selected C blocks only: out receives the blocks (i_q, j_q) concatenated, each r_i x t_j
 * row-major, value alpha * sum_k A_ik B_kj (no accumulation).  present[q] tells whether the block
 * belongs to the C-shape (an absent block is written as zeros). */
int oracle_bsmm_blocks(int64_t M, int64_t K, int64_t N, const int64_t* r, const int64_t* s,
                       const int64_t* t, const uint64_t* a_bits, const uint64_t* b_bits,
                       const double* A, const double* B, double alpha, int64_t nsel,
                       const int64_t* sel_i, const int64_t* sel_j, double* out, int32_t* present,
                       int extended, int ta, int tb) {
  problem p;
  if (setup(&p, M, K, N, r, s, t, a_bits, b_bits, ta, tb)) { teardown(&p); return -1; }
  int64_t* pos = (int64_t*)malloc((size_t)(nsel + 1) * sizeof(int64_t));
  if (!pos) { teardown(&p); return -1; }
  pos[0] = 0;
  for (int64_t q = 0; q < nsel; ++q) {
    if (sel_i[q] < 0 || sel_i[q] >= M || sel_j[q] < 0 || sel_j[q] >= N) { free(pos); teardown(&p); return -2; }
    pos[q + 1] = pos[q] + r[sel_i[q]] * t[sel_j[q]];
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < nsel; ++q) {
    double* o = out + pos[q];
    present[q] = block_product(&p, A, B, sel_i[q], sel_j[q], o, extended);
    int64_t hw = r[sel_i[q]] * t[sel_j[q]];
    for (int64_t e = 0; e < hw; ++e) o[e] = alpha * o[e];
  }
  free(pos); teardown(&p);
  return 0;
}

/* One complex C block (interleaved, r_i x t_j) = sum over present k of op(A)_ik op(B)_kj, k
 * ascending, elements in i-k-j order; ca / cb conjugate the operand.  Returns presence. */
static int zblock_product(const problem* p, const double* A, const double* B, int ca, int cb,
                          int64_t i, int64_t j, double* out) {
  int64_t h = p->r[i], w = p->t[j];
  int present = 0;
  for (int64_t e = 0; e < 2 * h * w; ++e) out[e] = 0.0;
  for (int64_t k = 0; k < p->K; ++k) {
    int64_t ao = a_at(p, i, k), bo = b_at(p, k, j);
    if (ao < 0 || bo < 0) continue;
    present = 1;
    int64_t d = p->s[k];
    const double* a = A + 2 * ao;
    const double* b = B + 2 * bo;
    for (int64_t x = 0; x < h; ++x)
      for (int64_t y = 0; y < d; ++y) {
        int64_t ea = p->ta ? y * h + x : x * d + y;
        double ar = a[2 * ea], ai = ca ? -a[2 * ea + 1] : a[2 * ea + 1];
        for (int64_t z = 0; z < w; ++z) {
          int64_t eb = p->tb ? z * d + y : y * w + z;
          double br = b[2 * eb], bi = cb ? -b[2 * eb + 1] : b[2 * eb + 1];
          out[2 * (x * w + z)] += ar * br - ai * bi;
          out[2 * (x * w + z) + 1] += ar * bi + ai * br;
        }
      }
  }
  return present;
}

/* Complex product: C = alpha op(A) op(B) (+ C), A, B, C interleaved complex; op_a, op_b: 0 = as
 * is, 1 = transpose, 2 = adjoint (stored as for the transpose). */
int oracle_zbsmm(int64_t M, int64_t K, int64_t N, const int64_t* r, const int64_t* s,
                 const int64_t* t, const uint64_t* a_bits, const uint64_t* b_bits, const double* A,
                 const double* B, double alpha_re, double alpha_im, int accumulate, double* C,
                 int op_a, int op_b) {
  problem p;
  if (setup(&p, M, K, N, r, s, t, a_bits, b_bits, op_a != 0, op_b != 0)) { teardown(&p); return -1; }
  int64_t wn = words_of(N);
  uint64_t* c_bits = (uint64_t*)calloc((size_t)(M * wn > 0 ? M * wn : 1), sizeof(uint64_t));
  int64_t* c_off = (int64_t*)malloc((size_t)(M * N > 0 ? M * N : 1) * sizeof(int64_t));
  if (!c_bits || !c_off) { free(c_bits); free(c_off); teardown(&p); return -1; }
  shape_of_product(&p, c_bits);
  oracle_block_offsets(M, N, r, t, c_bits, c_off);
  int status = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < M * N; ++q) {
    int64_t i = q / N, j = q % N;
    int64_t co = c_off[q];
    if (co < 0) continue;
    int64_t hw = r[i] * t[j];
    double* tmp = (double*)malloc((size_t)(hw > 0 ? 2 * hw : 1) * sizeof(double));
    if (!tmp) { status = -1; continue; }
    zblock_product(&p, A, B, op_a == 2, op_b == 2, i, j, tmp);
    for (int64_t e = 0; e < hw; ++e) {
      double xr = tmp[2 * e], xi = tmp[2 * e + 1];
      double vr = alpha_re * xr - alpha_im * xi, vi = alpha_re * xi + alpha_im * xr;
      double* c = C + 2 * (co + e);
      c[0] = accumulate ? vr + c[0] : vr;
      c[1] = accumulate ? vi + c[1] : vi;
    }
    free(tmp);
  }
  free(c_bits); free(c_off); teardown(&p);
  return status;
}

/* Selected complex C blocks (alpha = 1, no accumulation), as oracle_bsmm_blocks. */
int oracle_zbsmm_blocks(int64_t M, int64_t K, int64_t N, const int64_t* r, const int64_t* s,
                        const int64_t* t, const uint64_t* a_bits, const uint64_t* b_bits,
                        const double* A, const double* B, int64_t nsel, const int64_t* sel_i,
                        const int64_t* sel_j, double* out, int32_t* present, int op_a, int op_b) {
  problem p;
  if (setup(&p, M, K, N, r, s, t, a_bits, b_bits, op_a != 0, op_b != 0)) { teardown(&p); return -1; }
  int64_t* pos = (int64_t*)malloc((size_t)(nsel + 1) * sizeof(int64_t));
  if (!pos) { teardown(&p); return -1; }
  pos[0] = 0;
  for (int64_t q = 0; q < nsel; ++q) {
    if (sel_i[q] < 0 || sel_i[q] >= M || sel_j[q] < 0 || sel_j[q] >= N) { free(pos); teardown(&p); return -2; }
    pos[q + 1] = pos[q] + 2 * r[sel_i[q]] * t[sel_j[q]];
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < nsel; ++q)
    present[q] = zblock_product(&p, A, B, op_a == 2, op_b == 2, sel_i[q], sel_j[q], out + pos[q]);
  free(pos); teardown(&p);
  return 0;
}

/* Dense packed A (ordinary layout) from a block-rank-sparse A: ranks[q] of the q-th present block
 * in row-major block order, 0 = dense.  Returns -1 for a negative rank. */
int oracle_lr_expand(int64_t M, int64_t K, const int64_t* r, const int64_t* s,
                     const uint64_t* a_bits, const int32_t* ranks, const double* A_lr,
                     double* A_dense) {
  int64_t q = 0, src = 0, dst = 0;
  for (int64_t i = 0; i < M; ++i)
    for (int64_t k = 0; k < K; ++k) {
      if (!bit_at(a_bits, K, i, k)) continue;
      int64_t h = r[i], d = s[k], rho = ranks[q++];
      if (rho < 0) return -1;
      if (rho == 0) {
        for (int64_t e = 0; e < h * d; ++e) A_dense[dst + e] = A_lr[src + e];
        src += h * d;
      } else {
        const double* u = A_lr + src;            /* h x rho */
        const double* v = A_lr + src + h * rho;  /* d x rho */
        for (int64_t x = 0; x < h; ++x)
          for (int64_t y = 0; y < d; ++y) {
            double acc = 0.0;
            for (int64_t l = 0; l < rho; ++l) acc += u[x * rho + l] * v[y * rho + l];
            A_dense[dst + x * d + y] = acc;
          }
        src += (h + d) * rho;
      }
      dst += h * d;
    }
  return 0;
}

/* Eq. 1: the number of SUMMA iterations issued at once on a P_row x P_col grid with K blocks
 * along the inner dimension: 2 when either grid dimension is below 2, K when both reach K, and
 * min(P_row, P_col) otherwise. */
int64_t oracle_concurrent_iterations(int64_t prow, int64_t pcol, int64_t K) {
  if (prow < 2 || pcol < 2) return 2;
  if (prow >= K && pcol >= K) return K;
  return prow < pcol ? prow : pcol;
}

/* Eq. 2: average memory (in elements) one process holds per SUMMA iteration: the A column panel
 * share M m k / P_row, the B row panel share N k n / P_col and the local result
 * M N m n / (P_row P_col). */
double oracle_memory_overhead(double M, double N, double m, double n, double k, double prow,
                              double pcol) {
  return M * m * k / prow + N * k * n / pcol + M * N * m * n / (prow * pcol);
}
