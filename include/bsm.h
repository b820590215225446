/*
 * bsm -- block-sparse matrix multiply with nonuniform, problem-given block sizes, on one
 * MI355X (gfx950).  C ABI.
 *
 * The operation (Calvin & Valeev, "Task-Based Algorithm for Matrix Multiplication", SC15):
 * SUMMA builds C = A B up from one rank-k update C_ij <- A_ik B_kj + C_ij per k (Sec. 2.1;
 * Alg. 1's local step C <- alpha A(*,k) B(k,*) + C).  The task-based form over-decomposes the
 * matrices into blocks of freely chosen sizes (Sec. 3.2), splits every update into a block
 * product and a reduction into C, and lets many k-iterations run at once (multiple issue, Eq. 1).  This
 * library executes that local multiply for block-sparse operands: for every (i, j) in the
 * C-shape  Chat_ij = OR_k (Ahat_ik AND Bhat_kj)
 *     C_ij = alpha * sum_{k : Ahat_ik and Bhat_kj} A_ik B_kj   (+ C_ij when accumulating).
 * Either operand may be read transposed (Sec. 2.1's SUMMA variants for products with A^T or B^T):
 * options trans_a / trans_b replace A by A^T and B by B^T in the formulas above; see Transposes.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Tilings   int64 vectors of block sizes: rows (M blocks), inner (K blocks, A's columns and B's
 *           rows), cols (N blocks).  Every size is in [1, 65535].
 * Shapes    bitmaps, row-major, each row padded to whole 64-bit words: bit (i, j) of an R x C
 *           shape is bit j % 64 of word i * ceil(C / 64) + j / 64.  Padding bits must be 0.
 * Tiles     the present blocks, packed in row-major block order (i, then j); each block is
 *           row-major with leading dimension equal to its own column count.  A block's offset is
 *           the number of elements of the present blocks before it.  The same layout holds for
 *           C, whose shape is Chat.
 * Transposes with trans_a, the caller's A is the K x M block matrix whose transpose is the
 *           product's left operand: its shape is given as stored (K x M bits), its tiles are its
 *           own present blocks packed in its own row-major block order, block (k, i) of s_k x r_i
 *           elements, and the product reads block (k, i) transposed as op(A)_ik.  Likewise with
 *           trans_b the caller's B is N x K, block (j, k) of t_j x s_k elements.  The tilings
 *           always describe the product (r, s, t as above).  A transposed operand is copied into
 *           the product's layout by a transposition pass on the stream before the tile kernels
 *           (in the FP32 and split-bf16 forms, inside the conversion pass they run anyway).
 * Memory    host arguments are copied before the call returns.  Device buffers (dA, dB, dC) are
 *           owned by the caller and must stay valid until the work queued on the stream is done.
 *           dA and dB may be the same buffer (C = A A); dC must not overlap either.
 * Streams   `stream` is a hipStream_t (NULL = the default stream); work is queued on it and the
 *           call returns without waiting.  A plan runs on one stream at a time.  A call that must
 *           replace a device table a queued launch may still read (new task order after
 *           bsm_plan_set_costs, new operand pointers of a batch or of a plan with k_split > 1)
 *           first waits for the work queued on `stream`.
 * Errors    every call returns a bsm_status; nothing is thrown across the ABI.  The text of the
 *           last failure on the calling thread is available from bsm_last_error().  Device faults
 *           appear as BSM_E_HIP at the next call that synchronises.  Every launch counts, per
 *           task, how often the task ran; the calls that synchronise and read results back
 *           (bsm_plan_verify, bsm_batch_verify, bsm_plan_timings, bsm_batch_timings) return
 *           BSM_E_STATE if any task ran a number of times other than the launches queued.
 */
#ifndef BSM_H
#define BSM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BSM_OK = 0,
  BSM_E_INVALID = -1,     /* malformed argument: null pointer, size out of range, padding bit set */
  BSM_E_MISMATCH = -2,    /* arguments disagree with each other or with the plan */
  BSM_E_NOMEM = -3,       /* host or device allocation failed, or a stated limit was exceeded */
  BSM_E_HIP = -4,         /* a HIP runtime call failed (text in bsm_last_error) */
  BSM_E_UNSUPPORTED = -5, /* no gfx950 device, or an option the library does not provide */
  BSM_E_STATE = -6        /* call out of order, e.g. timings requested but never recorded */
} bsm_status;

/* Arithmetic of the block products.  Sums across k-blocks are FP64 in every form. */
typedef enum {
  BSM_FP64 = 0,  /* FP64 MFMA, FP64 accumulation */
  BSM_FP32 = 1,  /* operands rounded to FP32, FP32 MFMA within a block product, FP64 across k */
  BSM_BF16X3 = 2 /* each operand split into three bf16 slices, the six slice products of order
                    <= 2 on bf16 MFMA with FP32 accumulation within a block product, FP64
                    across k */
} bsm_precision;

/* Element type of C (the k-window partial sums stay FP64 either way). */
typedef enum {
  BSM_OUT_F64 = 0, /* C holds FP64 elements */
  BSM_OUT_F32 = 1  /* C holds FP32 elements: alpha * sum (+ C) is formed in FP64, rounded once */
} bsm_out;

/* Element type of A, B and C.  Complex elements (Sec. 4.3 lists real and complex types as both
 * supported) are stored as two doubles each, real part first, offsets and sizes counted in complex
 * elements.  A complex product runs as the real product of embeddings: op(A)_ik becomes the real
 * block [[Re, -Im], [Im, Re]] (2 r_i x 2 s_k) and op(B)_kj the block [Re; Im] (2 s_k x t_j), so
 * that the real C block is [Re C_ij; Im C_ij]; an embedding pass before the tile kernels and a
 * complex epilogue (alpha, accumulation, interleaving) after them run on the same stream.  Every
 * precision form applies to the real product.  Complex block sizes are at most 32767 rows and
 * inner columns. */
typedef enum {
  BSM_REAL = 0,
  BSM_COMPLEX = 1
} bsm_elem;

/* How tasks are ordered (never changes the numbers). */
typedef enum {
  BSM_SCHED_FLOPS = 0, /* cost = flop count */
  BSM_SCHED_MLP = 1    /* cost = the learned model's prediction (set with bsm_plan_set_costmodel) */
} bsm_sched;

/* How the scheduler deals tasks to the 8 accelerator dies (XCDs, each with its own L2). */
typedef enum {
  BSM_ORDER_DEFAULT = 0,    /* BSM_ORDER_LPT for plans (and batches) of up to 8192 tasks, where the
                               schedule's tail decides the makespan, else BSM_ORDER_INTERLEAVE */
  BSM_ORDER_INTERLEAVE = 1, /* whole C blocks, in C-block order, each to the least-loaded XCD */
  BSM_ORDER_LOCALITY = 2,   /* C-block order cut into 8 runs of equal cost */
  BSM_ORDER_LPT = 3,        /* largest cost first, each task to the least-loaded XCD */
  BSM_ORDER_PATCH = 4       /* rectangles of patch_rows x patch_cols C blocks, each whole to the
                               least-loaded XCD, so that the tasks an XCD runs at the same time
                               share few A block rows and B block columns in its L2 */
} bsm_order;

typedef struct {
  int32_t precision;      /* bsm_precision */
  int32_t sched;          /* bsm_sched */
  int64_t k_window;       /* k-iterations in flight at once (multiple issue, Sec. 3.2): 0 = all K */
  int32_t record_timings; /* 1 = record each task's start/end clock for bsm_plan_timings */
  int32_t tile;           /* 0 = chosen by the library; otherwise a tile variant id (bsm_tile_*) */
  int32_t use_graph;      /* 1 = bsm_execute captures its launches into a hipGraph and replays it
                             while the operands, alpha and accumulate stay the same */
  int32_t out;            /* bsm_out: element type of C */
  int32_t order;          /* bsm_order */
  int32_t patch_rows;     /* BSM_ORDER_PATCH: C-block rows per patch, 0 = 4 */
  int32_t patch_cols;     /* BSM_ORDER_PATCH: C-block columns per patch, 0 = 8 */
  int32_t device_klists;  /* where C blocks' k-lists (their block triples) are built:
                              0 = on the host while they fit a host list of 2^28 triples, else on
                              the device; -1 = always on the host; 1 = always on the device; n >= 2
                              = always on the device, in batches of at most n triples (the device
                              buffer for them; the default batch is 2^27 triples, 2 GiB) */
  int32_t trans_a;        /* 1 = the product reads A^T: A is stored as the K x M block matrix
                             (see Transposes); 2 = the adjoint A^H (stored as for 1; the same as
                             1 for real elements); 0 = as is */
  int32_t trans_b;        /* the same for B: 1 = B^T, 2 = B^H, stored as the N x K block matrix */
  int32_t elem;           /* bsm_elem: element type of A, B and C */
  int32_t k_split;        /* reduction variant (Sec. 3.2 splits each update into a multiply and a
                             reduction into C; the tile kernels fuse the two, one task per C
                             sub-tile): n in 2..16 cuts every task's k-list into up to n pieces
                             of equal triple count that run as separate tasks, each writing FP64
                             partial sums, which a reduction pass adds in piece order; for products
                             whose C has too few tiles to fill the GPU.  -1 = n chosen by the
                             library (2048 / tasks, at most 16) for products with fewer than 1024
                             tasks, none otherwise; 0 or 1 = off.  Changes the summation order,
                             not which terms are summed.  Needs k_window 0 and host k-lists
                             (BSM_E_UNSUPPORTED otherwise for n >= 2; -1 then means off); batches
                             and bsm_execute_static take plans without it. */
  const char* tune_cache; /* NULL, or a file where bsm_autotune looks up and records its choices
                             (lines "signature variant"); the string is copied */
} bsm_options;

typedef struct {
  int64_t M, K, N;         /* block counts */
  int64_t a_blocks, b_blocks, c_blocks;
  int64_t a_elems, b_elems, c_elems; /* packed buffer sizes in elements */
  int64_t triples;         /* (i,k,j) with both A_ik and B_kj present */
  int64_t tasks;           /* work items the GPU executes (C sub-tiles) */
  double useful_flops;     /* 2 * sum over triples of r_i s_k t_j */
  int64_t workspace_bytes; /* device memory the plan holds besides the caller's buffers */
  int64_t k_windows;       /* launches per execute: ceil(K / k_window) */
  int32_t tile;            /* tile variant every task uses (variant id + 1), or 0 when the size
                              classes use different variants (bsm_plan_tile_classes) */
  int32_t out;             /* bsm_out: element type of C */
  int32_t device_klists;   /* 1: the k-lists are built on the device, batch by batch */
  int32_t elem;            /* bsm_elem; a_elems, b_elems, c_elems count elements of this type */
  int32_t k_split;         /* pieces per k-list (1 = the fused C-stationary tasks only) */
} bsm_plan_info;

typedef struct bsm_batch bsm_batch;

typedef struct bsm_plan bsm_plan;

/* Fill opt with the defaults: FP64 products and FP64 C, flop-count scheduling, the automatic task
 * order, all k-iterations in flight, no timings, library-chosen tiles, no graph, no tune cache. */
void bsm_options_default(bsm_options* opt);

/* Build a plan for C = alpha A B (+ C) over problem-given blocks of any size (Sec. 3.2's
 * over-decomposition; Fig. 3 splits one iteration into tasks, each producing one piece of the
 * process's part of C).  Host-only work: validates the tilings and shapes, forms the C-shape (the
 * boolean product of the two shapes), the packed offsets, the task list (each present C block,
 * cut into sub-tiles; its k-list = the k with A_ik and B_kj present, in ascending order) and the
 * task order.  When the k-lists are built on the device (option device_klists), the host keeps
 * only each C block's k-list length and summed inner size, counted from the shape words, plus
 * the offset tables, and the tasks are cut into batches whose triples fit the device buffer; each
 * execute then builds a batch's triples on the device right before the batch's tile launch.
 * Device memory is allocated at the first execute.  a_bits and b_bits are the shapes as stored:
 * M x K and K x N, or K x M with trans_a and N x K with trans_b.  All arguments are host memory
 * and are copied; opt may be NULL (defaults).  Errors: BSM_E_INVALID for a null pointer, a
 * negative count, a block size outside [1, 65535], a padding bit set or an unknown option;
 * BSM_E_NOMEM if the host runs out or a buffer exceeds 2^48 elements. */
bsm_status bsm_plan_create(bsm_plan** out, int64_t M, const int64_t* row_sizes, int64_t K,
                           const int64_t* inner_sizes, int64_t N, const int64_t* col_sizes,
                           const uint64_t* a_bits, const uint64_t* b_bits,
                           const bsm_options* opt);

/* Sizes and counts of a plan (host memory, no device work).  useful_flops is the work of the
 * rank-k updates C_ij <- A_ik B_kj + C_ij that the shapes call for (Sec. 2.1). */
bsm_status bsm_plan_query(const bsm_plan* plan, bsm_plan_info* info);

/* The C-shape Chat = OR_k (Ahat_ik AND Bhat_kj) as a bitmap (M * ceil(N/64) words, host memory,
 * caller-owned): the block sparsity the product of two block-sparse operands has (Sec. 1). */
bsm_status bsm_plan_c_shape(const bsm_plan* plan, uint64_t* c_bits);

/* Packed element offset of every C block, -1 for an absent block (M * N int64, host memory,
 * caller-owned). */
bsm_status bsm_plan_c_offsets(const bsm_plan* plan, int64_t* c_offsets);

/* C = alpha A B (+ C if accumulate), queued on `stream`: Alg. 1's local update
 * C <- alpha A(*,k) B(k,*) + C for every k-iteration, i.e. all the rank-k updates of Sec. 2.1,
 * with each C block reduced over its k-list in ascending k.  dA, dB: device pointers to the
 * packed FP64 tiles (a_elems, b_elems elements); dC: device pointer to the packed C tiles
 * (c_elems elements of the plan's output type).  With accumulate = 0 every element of C is
 * written (present blocks only); with accumulate = 1 C must hold the previous values.  dA may
 * equal dB.  Errors: BSM_E_INVALID for null pointers or overlapping C; BSM_E_UNSUPPORTED without
 * a gfx950 device; BSM_E_HIP if a launch fails.  On a complex plan alpha is real (see
 * bsm_execute_complex). */
bsm_status bsm_execute(bsm_plan* plan, double alpha, const double* dA, const double* dB,
                       void* dC, int accumulate, void* stream);

/* C = alpha op(A) op(B) (+ C) with complex alpha = alpha_re + i alpha_im, for a plan with complex
 * elements (Sec. 4.3's complex type); the same call as bsm_execute otherwise.  dA, dB: device
 * pointers to the packed complex tiles (a_elems, b_elems complex elements, two doubles each,
 * 16-byte aligned); dC: c_elems complex elements of the output type (complex FP64, or complex
 * FP32 with BSM_OUT_F32), aligned to its element.  The embedded operands and the real product's
 * C live in device memory the plan owns.  Errors: as bsm_execute; BSM_E_INVALID for misaligned
 * buffers; BSM_E_MISMATCH for a nonzero alpha_im on a real plan. */
bsm_status bsm_execute_complex(bsm_plan* plan, double alpha_re, double alpha_im, const double* dA,
                               const double* dB, void* dC, int accumulate, void* stream);

/* For callers that cannot allocate device memory (code under hipGraph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same product as bsm_execute, with the same kernels
 * and task order (so bitwise the same C), that allocates nothing.  Everything bsm_execute would
 * allocate on the device -- task list, k-list triples, split tables, converted FP32 / bf16-slice
 * operands, FP64 partial sums between k-windows -- is placed in one static device array of
 * 64 MiB that each GPU the library runs on holds until the process ends; the tables are copied in
 * from the plan's host copy at every call (queued on `stream`).  Nothing in it needs to start at
 * zero.  Calls on one GPU share that array: calls on the same stream run one after the other,
 * calls that overlap on different streams of one GPU race and give wrong results.  Execution
 * counters and per-task clocks are not kept (bsm_plan_verify does not cover these calls), and the
 * plan's graph option is ignored.  Errors: as bsm_execute; BSM_E_NOMEM (checked before any device
 * work) if the plan needs more than the 64 MiB, with the size in bsm_last_error();
 * BSM_E_UNSUPPORTED for a plan whose k-lists are built on the device or a plan with complex
 * elements. */
bsm_status bsm_execute_static(const bsm_plan* plan, double alpha, const double* dA,
                              const double* dB, void* dC, int accumulate, void* stream);

/* Waits for `stream`, then checks that every task of the plan ran once per k-window of every
 * execute queued since the task list was last (re)uploaded.  BSM_E_STATE names the first task
 * that did not; BSM_E_HIP reports a device fault. */
bsm_status bsm_plan_verify(bsm_plan* plan, void* stream);

/* Fault injection for tests of the checks above: every later launch of the plan leaves task
 * `task` out (its workgroup returns at once; C keeps its old values there), -1 = none. */
bsm_status bsm_plan_debug_skip_task(bsm_plan* plan, int64_t task);

/* Per-task timings of the last execute of a plan created with record_timings = 1 (waits for
 * `stream` and checks the execution counters as bsm_plan_verify does).  The recorded times are
 * the training data of the learned cost model that orders tasks for dynamic scheduling (Sec. 3.2
 * leaves ordering to the runtime; Sec. 4.4 shows the block-level imbalance it has to absorb).  n must equal the plan's task count.  features (n x 5 floats, host; may be NULL)
 * receives each task's cost-model features: log h, log w, log (summed inner size of its k-list),
 * log (number of k-list blocks), k-list density (summed inner size / total inner size);
 * seconds (n floats, host; may be NULL) the task's duration on the device clock.
 * Errors: BSM_E_STATE if no timed execute has run, BSM_E_MISMATCH for a wrong n. */
bsm_status bsm_plan_timings(bsm_plan* plan, float* features, float* seconds, int64_t n,
                            void* stream);

/* The cost-model features of every task in the current task order (n x 5 floats, host; n = task
 * count): log h, log w, log (summed inner size of the k-list), log (number of k-list blocks),
 * k-list density.  Host-only. */
bsm_status bsm_plan_features(const bsm_plan* plan, float* features, int64_t n);

/* Re-order and re-bin the tasks by the given per-task costs (n floats, host, >= 0, in the current
 * task order; e.g. a cost model's predictions).  Only the schedule changes: every task still runs
 * once and C is bitwise the same.  The new order is uploaded at the next execute, after the work
 * queued on that execute's stream has finished. */
bsm_status bsm_plan_set_costs(bsm_plan* plan, const float* costs, int64_t n);

/* Autotuner.  C blocks fall into four size classes by their larger size (<= 32, <= 64, <= 128,
 * more); each class has its own tile variant, and the tasks of one variant are launched together.
 * For every class that carries work (most work first) every variant of the plan's precision form
 * is timed with the other classes fixed (one warm-up and 5 timed runs of the whole product on the
 * given operands; C is overwritten with A B), and the fastest is kept.  *chosen (may be NULL)
 * receives the variant id + 1 if all classes ended on one variant, else 0.  When the plan's
 * tune_cache option names a file, choices are looked up there by a workload signature first and
 * appended after tuning.  Synchronises `stream`.  (The paper's performance rests on the block
 * kernel, Sec. 4.3; this picks its tile shape per block size.) */
bsm_status bsm_autotune(bsm_plan* plan, const double* dA, const double* dB, void* dC,
                        void* stream, int32_t* chosen);

/* The tile variant (id + 1) of each of the four size classes (writes min(cap, 4) entries). */
bsm_status bsm_plan_tile_classes(const bsm_plan* plan, int32_t* variants, int32_t cap);

/* Set the tile variant (id + 1) of each of the four size classes (4 entries, host) and re-cut the
 * tasks (flop-count order).  Only the tiling changes; results stay within the form's gate. */
bsm_status bsm_plan_set_tile_classes(bsm_plan* plan, const int32_t* variants);

/* Release the plan (waits for its device work first).  NULL is accepted. */
bsm_status bsm_plan_destroy(bsm_plan* plan);

/* ---- block-rank-sparse left operand -----------------------------------------------------------
 * Sec. 1 names block-rank sparsity (blocks of low rank, as in hierarchical matrices) as the data
 * sparsity the task formulation is a step towards.  Here a present block of A is either dense or
 * stored as factors A_ik = U V^T, U r_i x rho and V s_k x rho, both row-major, U first.  The
 * caller's A buffer holds the present blocks in row-major block order, r_i s_k elements for a
 * dense block and (r_i + s_k) rho for a factored one; a_ranks[q] is the rank of the q-th present
 * block (0 = dense).  B and C keep the ordinary layout; C's shape is the C-shape of A B.
 *
 * The product runs as two ordinary products on the library's kernels (same precision forms):
 *   stage 1  W_(ik)j = V_ik^T B_kj for every factored (i,k) and present B_kj;
 *   stage 2  C = alpha [A_dense | U] [B ; W] (+ C), the inner dimension extended by one block of
 *            size rho per factored block,
 * after staging passes on the stream (dense blocks and U factors gathered, V factors transposed,
 * B copied in front of W) into device memory the plan owns.  A factored block therefore costs
 * 2 rho (s_k + r_i) t_j flops per present B_kj instead of 2 r_i s_k t_j. */
typedef struct bsm_lr_plan bsm_lr_plan;

typedef struct {
  int64_t M, K, N;
  int64_t a_blocks;         /* present blocks of A */
  int64_t factored_blocks;  /* of which stored as U V^T */
  int64_t a_elems;          /* the caller's A buffer (factors of factored blocks) */
  int64_t b_elems;
  int64_t c_blocks, c_elems;
  int64_t tasks;            /* tile-kernel tasks of both stages */
  int64_t workspace_bytes;  /* device memory the plan holds besides the caller's buffers */
  double useful_flops;      /* flops of both stages */
  double dense_flops;       /* flops of the same product with every block of A dense */
} bsm_lr_info;

/* Plan C = alpha A B (+ C) with a block-rank-sparse A (host work only; arguments copied).
 * a_ranks: one int32 per present A block in row-major block order, in [0, 65535].  opt as for
 * bsm_plan_create (the output type, precision form, order, graph option apply to both stages);
 * complex elements and transposed operands give BSM_E_UNSUPPORTED.  Errors: as bsm_plan_create. */
bsm_status bsm_lr_plan_create(bsm_lr_plan** out, int64_t M, const int64_t* row_sizes, int64_t K,
                              const int64_t* inner_sizes, int64_t N, const int64_t* col_sizes,
                              const uint64_t* a_bits, const int32_t* a_ranks,
                              const uint64_t* b_bits, const bsm_options* opt);

bsm_status bsm_lr_plan_query(const bsm_lr_plan* plan, bsm_lr_info* info);

/* Packed element offset of every C block, -1 for an absent block (M * N int64, host memory). */
bsm_status bsm_lr_plan_c_offsets(const bsm_lr_plan* plan, int64_t* c_offsets);

/* Queue the staging passes and both stages on `stream`.  dA: the caller's block-rank-sparse A
 * (a_elems FP64), dB: packed B, dC: packed C of the plan's output type.  Errors: as bsm_execute. */
bsm_status bsm_lr_execute(bsm_lr_plan* plan, double alpha, const double* dA, const double* dB,
                          void* dC, int accumulate, void* stream);

/* bsm_plan_verify for both stages. */
bsm_status bsm_lr_plan_verify(bsm_lr_plan* plan, void* stream);

/* Waits for the device, then frees the plan; NULL is ignored. */
bsm_status bsm_lr_plan_destroy(bsm_lr_plan* plan);

/* ---- block-sparse tensor contraction -----------------------------------------------------------
 * The paper's title and Sec. 1 present the block-sparse matrix product as a step towards
 * block-sparse tensor computing.  A block-sparse tensor of order d (1..8) has a tiling per mode and
 * a block shape over its block grid; its present blocks are packed in row-major order over the
 * grid (last mode fastest), each block dense and row-major over its modes.  Modes carry integer
 * labels.  C = alpha contract(A, B) (+ C): a label shared by A and B and absent from C is summed
 * over (its tilings must agree); every label of C comes from exactly one of A and B (labels in A,
 * B and C, or summed labels of one operand only, give BSM_E_UNSUPPORTED).  The contraction runs
 * as a block-sparse matrix product of the matricized operands (free modes of A in C's order x
 * contracted modes in A's order, times contracted x free modes of B in C's order); a permutation
 * pass per operand brings it into that order unless its mode order already is, and one brings C
 * into its mode order unless C lists A's free modes before B's.  Matricized blocks must stay
 * within 65535 rows and columns. */
typedef struct {
  int32_t order;           /* modes, 1..8 */
  const int32_t* modes;    /* label of each mode */
  const int64_t* nblocks;  /* blocks along each mode */
  const int64_t* sizes;    /* block sizes, mode after mode (sum of nblocks entries) */
  const uint64_t* bits;    /* block shape: bit q (word q / 64, bit q % 64) = the block with
                              row-major flattened grid index q; ceil(grid / 64) words */
} bsm_tensor;

typedef struct bsm_tc_plan bsm_tc_plan;

typedef struct {
  int64_t M, K, N;             /* block counts of the matricized product */
  int64_t a_blocks, b_blocks, c_blocks;
  int64_t a_elems, b_elems, c_elems;
  int64_t tasks;
  int64_t workspace_bytes;
  double useful_flops;         /* 2 x (elements of each contributing block pair product) */
  int32_t permute_a, permute_b, permute_c;  /* 1: that operand goes through a permutation pass */
} bsm_tc_info;

/* Plan a contraction (host work; descriptors and labels are copied).  C's tilings and block shape
 * follow from A and B.  opt as for bsm_plan_create (precision form, output type, order, graph);
 * complex elements and the trans options give BSM_E_UNSUPPORTED.  Errors: BSM_E_INVALID for a
 * malformed descriptor, BSM_E_MISMATCH for contracted modes with different tilings. */
bsm_status bsm_tc_plan_create(bsm_tc_plan** out, const bsm_tensor* A, const bsm_tensor* B,
                              int32_t c_order, const int32_t* c_modes, const bsm_options* opt);

bsm_status bsm_tc_plan_query(const bsm_tc_plan* plan, bsm_tc_info* info);

/* C's block shape over its flattened grid (ceil(grid / 64) words, host memory). */
bsm_status bsm_tc_plan_c_shape(const bsm_tc_plan* plan, uint64_t* c_bits);

/* Queue the permutation passes and the product on `stream`.  dA, dB: packed FP64 tensors; dC: C
 * packed in its own mode order, of the plan's output type.  Errors: as bsm_execute. */
bsm_status bsm_tc_execute(bsm_tc_plan* plan, double alpha, const double* dA, const double* dB,
                          void* dC, int accumulate, void* stream);

/* bsm_plan_verify for the product. */
bsm_status bsm_tc_plan_verify(bsm_tc_plan* plan, void* stream);

/* Waits for the device, then frees the plan; NULL is ignored. */
bsm_status bsm_tc_plan_destroy(bsm_tc_plan* plan);

/* ---- batches: many independent products in one launch ---------------------------------------
 * Several matrix multiplications overlapped in one execution (Sec. 1 names the overlap of the
 * multiplications of one expression as a motivation of the task formulation).  A batch
 * concatenates the tasks of n plans (same precision, k_window 0) into one task
 * list and one schedule; bsm_batch_execute captures every member's operand conversion plus the
 * tile-kernel launches over all tasks (one per tile variant in use) into a hipGraph and replays it
 * while the operand pointers, alphas and accumulate stay the same.  The plans must outlive the batch and must not run
 * elsewhere while the batch executes.  An FP64 plan may appear more than once (each entry is a
 * product with its own operands); an FP32 or split-bf16 plan only once, since it converts its
 * operands into buffers it owns (BSM_E_INVALID otherwise).  Members have real elements
 * (BSM_E_UNSUPPORTED for a complex plan). */
bsm_status bsm_batch_create(bsm_batch** out, bsm_plan* const* plans, int64_t n);

/* Task count, total useful flops and tile variant (id + 1, or 0 when the tasks mix variants) of a
 * batch (any pointer may be NULL). */
bsm_status bsm_batch_query(const bsm_batch* batch, int64_t* tasks, double* useful_flops,
                           int32_t* tile);

/* C_q = alphas[q] A_q B_q (+ C_q) for every member q.  alphas, dA, dB, dC: host arrays of n
 * entries (alphas may be NULL = all 1); the pointers they hold are device buffers as for
 * bsm_execute. */
bsm_status bsm_batch_execute(bsm_batch* batch, const double* alphas, const double* const* dA,
                             const double* const* dB, void* const* dC, int accumulate,
                             void* stream);

/* As bsm_plan_verify, over the batch's task list (one execution per bsm_batch_execute). */
bsm_status bsm_batch_verify(bsm_batch* batch, void* stream);

/* Per-task features and durations of the last batch execute (members created with
 * record_timings = 1), as bsm_plan_timings; n = the batch's task count. */
bsm_status bsm_batch_timings(bsm_batch* batch, float* features, float* seconds, int64_t n,
                             void* stream);

/* Re-order and re-bin the batch's tasks by per-task costs, as bsm_plan_set_costs. */
bsm_status bsm_batch_set_costs(bsm_batch* batch, const float* costs, int64_t n);

/* Autotuner over the whole batch, per size class as bsm_autotune (every member is re-cut with the
 * chosen class variants; the batch's tune cache is its first member's). */
bsm_status bsm_batch_autotune(bsm_batch* batch, const double* const* dA, const double* const* dB,
                              void* const* dC, void* stream, int32_t* chosen);

/* The tile variant (id + 1) of each size class of the batch (writes min(cap, 4) entries). */
bsm_status bsm_batch_tile_classes(const bsm_batch* batch, int32_t* variants, int32_t cap);

bsm_status bsm_batch_destroy(bsm_batch* batch);

/* ---- learned task cost model ---------------------------------------------------------------------
 * A small fully connected network (5 -> 32 -> 32 -> 1, ReLU, FP32) predicts a task's log run time
 * from its features (bsm_plan_features).  It is trained on the device (forward, backward, Adam)
 * from timings the multiply records itself (record_timings, bsm_plan_timings), and the scheduler
 * then bins and orders tasks by exp(prediction) instead of by flop count.  Only the schedule
 * changes; C is bitwise the same.  Parameter layout: W1 (32 x 5, row-major), b1 (32), W2 (32 x 32,
 * row-major), b2 (32), w3 (32), b3 (1).  Inputs are standardised with per-feature means and
 * standard deviations, and the output de-standardised, with statistics of the training set
 * ("norm12": 5 feature means, 5 feature scales, target mean, target scale). */
typedef struct bsm_costmodel bsm_costmodel;

/* New model with He-uniform initial weights drawn from splitmix64(seed, index), zero biases and
 * identity normalisation.  Host-only until first used. */
bsm_status bsm_costmodel_create(bsm_costmodel** out, uint64_t seed);
int64_t bsm_costmodel_param_count(void);
/* Copy the parameters (n = bsm_costmodel_param_count(), may be NULL) and/or the 12 normalisation
 * values (may be NULL) out of / into the model (host arrays). */
bsm_status bsm_costmodel_params(const bsm_costmodel* m, float* params, int64_t n, float* norm12);
bsm_status bsm_costmodel_set_params(bsm_costmodel* m, const float* params, int64_t n,
                                    const float* norm12);
/* Train on n samples (host: features n x 5, log run times n): set the normalisation from the
 * samples, then `epochs` passes of mini-batches of `batch` samples in index order, one Adam step
 * (lr, beta1 0.9, beta2 0.999, eps 1e-8) per mini-batch, all on the device.  *final_loss (may be
 * NULL) receives the mean squared error over all samples in standardised units.  Synchronises. */
bsm_status bsm_costmodel_train(bsm_costmodel* m, const float* features, const float* log_seconds,
                               int64_t n, int64_t epochs, int64_t batch, float lr,
                               float* final_loss, void* stream);
/* Predicted log run times (host in, host out; computed on the device).  Synchronises. */
bsm_status bsm_costmodel_predict(bsm_costmodel* m, const float* features, int64_t n,
                                 float* log_seconds, void* stream);
/* Persist / restore parameters, normalisation and Adam state (training can resume). */
bsm_status bsm_costmodel_save(const bsm_costmodel* m, const char* path);
bsm_status bsm_costmodel_load(bsm_costmodel** out, const char* path);
bsm_status bsm_costmodel_destroy(bsm_costmodel* m);
/* Re-bin and re-order the tasks by the model's predictions (S4 with the learned cost). */
bsm_status bsm_plan_set_costmodel(bsm_plan* plan, bsm_costmodel* model, void* stream);
bsm_status bsm_batch_set_costmodel(bsm_batch* batch, bsm_costmodel* model, void* stream);

/* The network's own arithmetic on device buffers, without normalisation: y = f(x) for n samples
 * (x: n x 5); the mean squared error over n samples and its gradient (d_loss may be NULL;
 * synchronises); one Adam step over n parameters (step = 1, 2, ...). */
bsm_status bsm_mlp_forward(const float* d_params, const float* d_x, int64_t n, float* d_y,
                           void* stream);
bsm_status bsm_mlp_loss_grad(const float* d_params, const float* d_x, const float* d_t, int64_t n,
                             float* d_grad, float* d_loss, void* stream);
bsm_status bsm_adam_step(float* d_params, const float* d_grad, float* d_m, float* d_v, int64_t n,
                         int64_t step, float lr, float beta1, float beta2, float eps, void* stream);

/* Eq. 1: how many SUMMA iterations are issued at once on a P_row x P_col process grid with K
 * inner blocks: 2 if either grid dimension is below 2, K if both are at least K, else
 * min(P_row, P_col). */
int64_t bsm_concurrent_iterations(int64_t p_row, int64_t p_col, int64_t K);

/* The tile variants of the FP64 and FP32 forms: variant v (option tile = v + 1) computes C
 * sub-tiles of at most tm[v] x tn[v] elements per workgroup.  Writes up to `cap` entries (either array may be
 * NULL) and returns the number of variants. */
int32_t bsm_tile_variants(int32_t* tm, int32_t* tn, int32_t cap);

/* The same for the split-bf16 form's tile variants. */
int32_t bsm_bf16_tile_variants(int32_t* tm, int32_t* tn, int32_t cap);

/* Text of the last error on the calling thread ("" if none). */
const char* bsm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BSM_H */
