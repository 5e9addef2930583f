/*
 * spmm.h - block-sparse x dense matrix multiplication on AMD MI355X (gfx950).
 *
 * The operation is the SpMM of PopSparse (arXiv 2303.16999, Section 3):
 *
 *     Y = (M o W) * X,    M[i][j] = M_hat[i / b][j / b]
 *
 * W is m x k and keeps only the b x b blocks whose entry of the block mask
 * M_hat (ceil(m/b) x ceil(k/b)) is one; X is k x n and dense; Y is m x n and
 * dense. m and k are the feature sizes, n the batch size, b the block size
 * (Section 3). Two modes follow Section 3.2 and 3.3:
 *
 *   static   the pattern is known ahead of time; a plan is built once and the
 *            values are supplied later (Section 3.2);
 *   dynamic  only a maximum number of nonzero blocks is fixed; the pattern and
 *            values arrive with every call (Section 3.3, Appendix A.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns spmm_status_t. Nothing throws across the ABI.
 *   spmm_last_error() returns a thread-local message for the last non-OK
 *   status returned on the calling thread.
 * - Argument errors are detected on the host and returned before any work is
 *   enqueued.
 * - Dense matrices are row-major with a leading dimension in elements
 *   (ldx >= n, ldy >= n). X and Y base addresses must be 16-byte aligned and
 *   ld * element_size must be a multiple of 16 bytes. Only columns [0, n) are
 *   read from X and written to Y. Y must not overlap X.
 * - "_dev" pointers are device memory (hipMalloc or a torch CUDA tensor),
 *   "_host" pointers are host memory. The library never frees caller memory.
 * - stream is a hipStream_t passed as void* (NULL = the default stream). Run
 *   calls only enqueue work on that stream and return without synchronising;
 *   X and Y are borrowed until that work completes.
 * - beta = 0: Y is fully overwritten; rows without blocks become +0.0.
 * - m and k need not be multiples of b: edge blocks are stored as full b x b
 *   blocks and their part outside the matrix is ignored, even if it holds
 *   non-finite values.
 * - Accumulation is in FP32 for every dtype; the output is rounded to Y's
 *   dtype to nearest-even. Results are bitwise reproducible run to run.
 *
 * Supported dtype triples (w, x, y):
 *   (F32, F32, F32)
 *   (F16, F16, F16 | F32)
 *   (BF16, BF16, BF16 | F32)
 *   (FP8_E4M3, F16 | BF16, same as x | F32)   one FP32 scale per block
 * FP8_E4M3 is the OCP E4M3FN format (bias 7, max 448, no infinities). A block
 * element stands for decode(code) * scale[block].
 *
 * Block sizes: b in {1, 4, 8, 16, 32}.
 */
#ifndef SPMM_H_
#define SPMM_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPMM_OK = 0,
  SPMM_ERR_INVALID_ARG = 1,  /* bad pointer, size, alignment, leading dimension */
  SPMM_ERR_UNSUPPORTED = 2,  /* valid request this build does not implement    */
  SPMM_ERR_CAPACITY = 3,     /* dynamic nnz above the declared maximum          */
  SPMM_ERR_BAD_INDEX = 4,    /* dynamic block index outside the block grid      */
  SPMM_ERR_OOM = 5,          /* device allocation failed                        */
  SPMM_ERR_HIP = 6,          /* a HIP runtime call failed                       */
  SPMM_ERR_REJECTED = 7      /* serving admission refused the request           */
} spmm_status_t;

typedef enum { SPMM_F32 = 0, SPMM_F16 = 1, SPMM_BF16 = 2, SPMM_FP8_E4M3 = 3 } spmm_dtype_t;

/* Plan options. Zero-initialise and set what you need.
 *   group_rows  block rows per row group of the plan (0 = choose);
 *   num_panels  contiguous ranges of row groups balanced by cost (0 = one
 *               group per panel);
 *   n_hint      expected batch size n, used only to choose group_rows;
 *   variant     tile variant of the compute kernel (0 = choose: the
 *               autotuner's result for this n class if there is one, else a
 *               measurement on the first run, else a rule on n; see the
 *               autotuner below). A variant is ns + 256 * form. ns, the tile
 *               width: for b = 16/32 with 16-bit X, 2, 4 or 8 column tiles of
 *               16 per wave; for b = 1/4/8 with 16-bit X, 4 or 8 columns per
 *               lane; 0 = the rule on n. form: 0 = the rule, 1 = the plain
 *               kernel, 2 = the plan's other kernel where it has one (the
 *               software-pipelined row kernel for b = 16/32 with W in the X
 *               type and no split rows; the LDS-staged kernel for b = 1, 4
 *               and 8 with W in the X type), else the plain one; 3 = the dense GEMM on
 *               the plan's dense copy (needs dense_dispatch that keeps one);
 *               4 = the row kernel with every block row split over the four
 *               waves of a workgroup, partial sums added in wave order (b =
 *               16 with 16-bit X; the rule takes it for launches too small to
 *               fill the chip with one wave per row, SPMM_SPLIT_ALL=0/1
 *               forces it; it sums in another order than forms 1 and 2);
 *               5 = dynamic calls only: form 4's product with the encoding
 *               in the same launch (a plan option rejects it).
 *               Other kernels have one variant and ignore it.
 *   dense_dispatch  static plans with W in the 16-bit X type and Y in it or
 *               FP32 (dynamic handles ignore it). 0 = never dense. 1 = ask the
 *               speedup model (spmm_speedup_model at feature size sqrt(m k),
 *               the plan's density and b) when the plan is built; where it
 *               predicts the sparse product slower than dense (ratio < 1),
 *               the plan keeps a dense copy of M o W (m x k, built by
 *               spmm_plan_set_values) and runs with variant 0 use a library
 *               GEMM on it, unless the autotuner measures a sparse variant
 *               faster. 2 = always keep the copy (runs still follow the model
 *               or the tuner). A fused ReLU (grouped and serving launches)
 *               always takes the sparse kernels. The dense GEMM's summation
 *               order is the library's: its results are within the FP32
 *               accumulation bound but not promised bit for bit from run to
 *               run, unlike the sparse kernels'. */
typedef struct {
  int32_t group_rows;
  int32_t num_panels;
  int32_t n_hint;
  int32_t variant;
  int32_t dense_dispatch;
} spmm_plan_opts;

typedef struct spmm_plan_s* spmm_plan_t;
typedef struct spmm_dyn_s* spmm_dyn_t;
typedef struct spmm_group_s* spmm_group_t;
typedef struct spmm_srv_s* spmm_srv_t;

/* Message for the last non-OK status on this thread ("" if none). The pointer
 * stays valid until the next library call on the same thread. */
const char* spmm_last_error(void);

/* ------------------------------------------------------------------ static mode
 * Static sparsity, Section 3.2: the pattern is known when the plan is built
 * (the paper's compile time); values are provided afterwards and reordered
 * once into the plan's layout.
 *
 * spmm_plan_static builds the plan on the current HIP device from a host
 * block mask: block_mask_host is uint8 [ceil(m/b)][ceil(k/b)] row-major,
 * nonzero = block present. The block-CSR (row_ptr, col_idx), the row groups
 * and the cost-balanced panels are computed by HIP kernels; the call
 * synchronises before returning. opts may be NULL.
 * b = 64 (beyond the paper's sweep) runs as 4 x 4 MFMA tiles of 16 (the
 * four waves of a workgroup take a block row's four row tiles) and needs
 * FP16 or BF16 X; its block rows are never split.
 * Errors: INVALID_ARG (m, k < 1, b not in {1,4,8,16,32,64}, NULL pointers),
 * UNSUPPORTED (dtype triple, b = 64 with FP32 X), OOM, HIP. On error *out is
 * NULL. */
spmm_status_t spmm_plan_static(int64_t m, int64_t k, int32_t b, const uint8_t* block_mask_host,
                               spmm_dtype_t w, spmm_dtype_t x, spmm_dtype_t y,
                               const spmm_plan_opts* opts, spmm_plan_t* out);

/* Blocked-ELL input. The paper's GPU comparison sets aside cuSPARSE's
 * blocked-ELL format, whose rows each list a fixed number of block-column
 * indices with -1 marking an empty slot (Appendix B; Section 5 notes it as the
 * FP16-capable layout that needs explicit padding). spmm_plan_ell takes that
 * description: ell_cols_host is int32 [ceil(m/b)][ell_width] row-major, each
 * entry a block column in [0, ceil(k/b)) or -1; slots of a row may come in
 * any order, but a column may appear only once per row. The result is the
 * plan spmm_plan_static builds from the equivalent mask (same kernels, same
 * results), which also remembers the slot of each block. b and opts as for
 * spmm_plan_static. Synchronises.
 * Errors: INVALID_ARG (sizes, NULL, index outside [-1, ceil(k/b)), repeated
 * column in a row), UNSUPPORTED, OOM, HIP.
 *
 * spmm_plan_set_values_ell: values in slot order, [ceil(m/b)][ell_width] blocks
 * of b x b (row-major inside a block); empty slots are not read. FP8 weights
 * take FP32 scales [ceil(m/b)][ell_width]. Gathers into the plan's order on
 * `stream` through a temporary buffer and synchronises `stream` before
 * returning. Errors: INVALID_ARG (NULL, plan not built from ELL), OOM, HIP. */
spmm_status_t spmm_plan_ell(int64_t m, int64_t k, int32_t b, int32_t ell_width, const int32_t* ell_cols_host,
                            spmm_dtype_t w, spmm_dtype_t x, spmm_dtype_t y, const spmm_plan_opts* opts,
                            spmm_plan_t* out);
spmm_status_t spmm_plan_set_values_ell(spmm_plan_t plan, const void* values_ell_dev, const float* scales_ell_dev,
                                       void* stream);

/* Copies the nonzero block values into plan-owned device memory (the plan
 * keeps them resident; the caller may free its buffer once the copy on
 * `stream` has completed). values_dev holds nnzb blocks of b x b elements of
 * dtype w, row-major inside each block, in block-CSR order (block rows in
 * ascending order, columns ascending within a row: the row-major order of the
 * mask). block_scales_dev: FP32 [nnzb] for FP8 weights, NULL otherwise.
 * Must be called before spmm_run_static; may be called again to replace the
 * values (stream-ordered with later runs on the same stream). */
spmm_status_t spmm_plan_set_values(spmm_plan_t plan, const void* values_dev,
                                   const float* block_scales_dev, void* stream);

/* Y = (M o W) * X with the plan's pattern and values. X: k x n of dtype x,
 * Y: m x n of dtype y. n = 0 is a no-op returning OK. The first run of a plan
 * whose variant is 0, for an n class with no tuned entry, runs the autotuner
 * on these operands (spmm_autotune_static; it synchronises `stream`), unless
 * SPMM_AUTOTUNE=0 or `stream` is capturing a graph: then the rule on n runs.
 * Y holds the product either way. A plan that cuts long rows into pieces
 * (spmm_plan_info) keeps a workspace for them, allocated on the first run
 * with more columns than it holds (after a device synchronisation); a run
 * captured in a graph that would need it to grow splits those rows over one
 * workgroup each instead, which may change the last bits. Runs of one such
 * plan share its workspace: runs that overlap in time (different streams or
 * threads) race and must be ordered by the caller.
 * Errors: INVALID_ARG (values not set, NULL, ld < n, alignment), HIP. */
spmm_status_t spmm_run_static(spmm_plan_t plan, int64_t n, const void* X, int64_t ldx,
                              void* Y, int64_t ldy, void* stream);

/* Plan facts: nonzero blocks, block rows per group, number of groups, panels,
 * and the number of block rows the row-wise kernel (b = 16, 16-bit X)
 * splits over the four waves of a workgroup: rows with more than
 * max(64, 2 x the mean) blocks, found when the plan is built (Appendix A.2's
 * worst case is a partition whose nonzeros all sit in one row). Rows longer
 * than max(256, 2 x that limit) blocks can also be cut into pieces of at most
 * that many blocks, one workgroup each, where a run finds their lengths
 * widely spread or too few workgroups for the chip; a second launch on the
 * same stream adds the pieces' FP32 partial sums in piece order. Both
 * reductions are in a fixed order, so results stay bitwise reproducible (and
 * equal between spmm_run_static and spmm_group_run), but a dynamic call of
 * the same pattern, which never splits, may differ from it in the last bits.
 * The remaining rows are taken longest first where the pattern is skewed (a
 * row over twice the mean, or any split row), which changes no result. Any
 * pointer may be NULL. */
/* Dense dispatch facts: *predicted_speedup (may be NULL) receives the speedup
 * model's sparse/dense ratio for the plan's shape (0 for an empty pattern);
 * *has_dense (may be NULL) whether the plan keeps a dense copy of M o W.
 * Errors: INVALID_ARG (NULL plan). */
spmm_status_t spmm_plan_dispatch(spmm_plan_t plan, double* predicted_speedup, int32_t* has_dense);

/* Device memory the plan holds: *device_bytes (may be NULL) all of its
 * buffers (plan arrays, values, scales, split-row, piece and SDDMM task
 * lists, ELL slots, the dense copy, the piece workspace), *value_bytes (may be NULL) its one copy of the block
 * values and FP8 scales. Host bookkeeping only.
 * Errors: INVALID_ARG (NULL plan). */
spmm_status_t spmm_plan_memory(spmm_plan_t plan, int64_t* device_bytes, int64_t* value_bytes);

spmm_status_t spmm_plan_info(spmm_plan_t plan, int64_t* nnzb, int32_t* group_rows,
                             int32_t* num_groups, int32_t* num_panels, int32_t* num_split_rows);

/* Host copies of the plan arrays, for inspection and tests (Section 3.2: the
 * static partition of the known blocks):
 *   row_ptr   int32 [mb + 1], col_idx int32 [nnzb]: block-CSR, block rows
 *             ascending, columns ascending inside a row;
 *   panel_ptr int32 [num_panels + 1]: group indices, panels balanced by the
 *             cost blocks + rows of their groups;
 *   order     int32 [nnzb]: CSR positions listed group by group, inside a
 *             group by (block column, block row): the column-major walk of a
 *             group's blocks.
 * Any pointer may be NULL to skip that array. Synchronises the device. */
spmm_status_t spmm_plan_export(spmm_plan_t plan, int32_t* row_ptr, int32_t* col_idx,
                               int32_t* panel_ptr, int32_t* order);

spmm_status_t spmm_plan_destroy(spmm_plan_t plan);

/* ------------------------------------------------------------------ training-direction products
 * Differentiating Y = (M o W) X (Section 3; sparse training motivates the
 * paper, Section 1) gives the data gradient dX = (M o W)^T dY, the same
 * block structure transposed, and the weight gradient dW = (dY X^T) o M, a
 * product sampled at the mask's blocks.
 *
 * spmm_plan_transpose builds, on the current device, the plan of W^T (k x m):
 * block (r, c) of W becomes block (c, r) with its values transposed. The
 * source plan must have values set; they are copied (later set_values calls
 * on the source do not reach the transposed plan). spmm_run_static on the
 * result computes (M o W)^T dY. opts as for spmm_plan_static. Synchronises.
 * Errors: INVALID_ARG (NULL, values not set), OOM, HIP.
 *
 * spmm_sddmm: G[e] = dY[rows of r] * X[rows of c]^T for every nonzero block
 * e = (r, c) of the plan, in its block-CSR order (the order of
 * spmm_plan_set_values). dY is m x n with the plan's y dtype, X is k x n with
 * its x dtype (both FP16 or both BF16), row-major, leading dimensions lddy and
 * ldx; G is FP32 [nnzb][b][b] row-major on the device (caller-owned). Rows
 * and columns of edge blocks outside m x k come out 0. b = 1, 4, 8, 16 or
 * 32. FP32 accumulation over n. Where the mask is dense enough for its block
 * size (density at least 1/128, 1/32, 1/16, 3/16, 1/4 for b = 1, 4, 8, 16,
 * 32), the product is a library GEMM of all of dY X^T (FP32, in row panels of
 * at most 128 MiB that the plan keeps from its first use) and a gather of the
 * mask's blocks, else kernels that compute only the mask's blocks;
 * SPMM_SDDMM_DENSE=0/1 forces the choice. The two sum in different orders.
 * Calls of one plan share that panel: calls that overlap in time (different
 * streams or threads) race and must be ordered by the caller.
 * Errors: INVALID_ARG (NULL, ld < n, alignment), UNSUPPORTED (block size
 * 64, dtypes), HIP. */
spmm_status_t spmm_plan_transpose(spmm_plan_t plan, const spmm_plan_opts* opts, spmm_plan_t* out);
spmm_status_t spmm_sddmm(spmm_plan_t plan, int64_t n, const void* dY, int64_t lddy, const void* X, int64_t ldx,
                         float* G, void* stream);

/* ------------------------------------------------------------------ speedup model
 * Section 5 summarises the paper's static sweep by a power law: a static
 * sparse product beats dense where a m^alpha d^beta b^gamma > 1. This is the
 * same form refitted to this library's static kernels against dense FP16 GEMM
 * (both FP16, FLOPs of the nonzeros only, each best over n) on one MI355X:
 * m = k in 2^8 .. 2^13, b in {1, 4, 8, 16}, density 1/4 .. 1/32. *speedup
 * receives the predicted ratio for feature size m = k, density d (0 < d <= 1)
 * and block size b, for dispatching between a sparse and a dense product; it
 * interpolates the measured grid and is not meant beyond it. Pure host code.
 * Errors: INVALID_ARG (NULL, m < 1, b < 1, density outside (0, 1]). */
spmm_status_t spmm_speedup_model(int64_t m, double density, int32_t b, double* speedup);

/* ------------------------------------------------------------------ autotuner
 * The paper's planner fixes the partition of (m, k, n) from the matrix sizes
 * and the density ahead of time (Appendix A); the analogous choice here is the
 * compute kernel's variant (tile width and kernel form), and it is made by
 * measurement. spmm_autotune_static runs every candidate variant of the
 * plan's kernels on the caller's X and Y (n columns; Y receives the result),
 * times each with HIP events on `stream` (untimed warm-up runs, then five
 * interleaved rounds of one launch per candidate, the median kept), and
 * records the fastest for n's size class (the power of two at or above n) in
 * the plan and in a process-wide table keyed by (b, dtypes, density class =
 * round(-log2 d), n class, whether the plan keeps a dense copy). Plans with
 * variant 0 use that table. With the
 * environment variable SPMM_AUTOTUNE_CACHE naming a file, the table starts
 * from that file when it was written for the same device (architecture and
 * CU count) and HIP runtime, and every new entry rewrites it (JSON, through a
 * temporary file and a rename); an unreadable file is ignored.
 * Synchronises `stream`. *variant_out (may be NULL) receives the choice;
 * times_ms_out (may be NULL) receives, for tile widths 2, 4 and 8 in that
 * order, the best mean time over the kernel forms with that width, -1 where
 * there is none (forms without a width of their own, ns = 0, appear only in
 * spmm_autotune_static_all).
 * spmm_autotune_static_all: the same, reporting every candidate: variants and
 * times_ms (capacity >= 8 entries each) receive *count candidates and their
 * mean times, *best (may be NULL) the choice.
 * spmm_plan_variant: the variant a run with n columns uses now (0 = not tuned
 * for n's class: the next spmm_run_static tunes, or the rule on n).
 * spmm_autotune_clear: forgets the process-wide table (not the plans' own
 * choices, not the cache file, which is not read again in this process).
 * Errors: as spmm_run_static; INVALID_ARG for capacity < 8 or NULL outputs. */
spmm_status_t spmm_autotune_static(spmm_plan_t plan, int64_t n, const void* X, int64_t ldx, void* Y,
                                   int64_t ldy, void* stream, int32_t* variant_out, float* times_ms_out);
spmm_status_t spmm_autotune_static_all(spmm_plan_t plan, int64_t n, const void* X, int64_t ldx, void* Y,
                                       int64_t ldy, void* stream, int32_t capacity, int32_t* variants,
                                       float* times_ms, int32_t* count, int32_t* best);
spmm_status_t spmm_plan_variant(spmm_plan_t plan, int64_t n, int32_t* variant);
spmm_status_t spmm_autotune_clear(void);

/* ------------------------------------------------------------------ grouped launch
 * Many static products with different plans, column counts, X and Y in one
 * kernel launch: one workgroup per work unit of all the problems. This goes
 * beyond the paper, whose benchmarks run one product at a time and let n grow
 * to amortise overheads (Sections 4 and 5); here the columns of many small
 * products share one launch instead. Up to 28 problems travel in the kernel
 * arguments of one direct launch (with SPMM_GROUP_GRAPH=1 in the environment,
 * the call instead replays a captured one-node HIP graph after updating that
 * node's arguments and grid). Larger groups go through a ring of
 * four pinned host + device tables: the call copies its table and launches
 * on it, and waits on the host only when the slot it needs is still in use by
 * the call four before.
 *
 * spmm_group_create makes a handle for up to max_problems problems.
 * spmm_group_run: problem i computes Y[i] = (M o W)_plans[i] * X[i] with
 * n[i] columns (0 = skipped), leading dimensions ldx[i] and ldy[i], and
 * applies max(0, .) before rounding when relu is non-NULL and relu[i] != 0.
 * Every plan must have values set and share block size (16 or 32) and dtype
 * triple, with 16-bit W and X (FP8 weights: UNSUPPORTED). Each problem uses
 * the variant its plan holds for its n (fixed, tuned, else the rule; a
 * grouped launch never tunes), so its result equals, bit for bit, a
 * spmm_run_static of that plan that runs the same variant. The handle keeps
 * a workspace for plans that cut long rows into pieces, one range per
 * problem (a plan may appear several times), grown like a plan's. Calls on
 * one handle must not overlap on different streams.
 * Errors: INVALID_ARG (count > max_problems, NULL, alignment, ld < n, values
 * not set, mixed block size or dtypes), UNSUPPORTED, HIP. */
spmm_status_t spmm_group_create(int32_t max_problems, spmm_group_t* out);
spmm_status_t spmm_group_run(spmm_group_t g, int32_t count, const spmm_plan_t* plans, const int64_t* n,
                             const void* const* X, const int64_t* ldx, void* const* Y, const int64_t* ldy,
                             const uint8_t* relu, void* stream);
spmm_status_t spmm_group_destroy(spmm_group_t g);

/* ----------------------------------------------------------------- dynamic mode
 * Dynamic sparsity, Section 3.3 and Appendix A.2: only the maximum number of
 * nonzero blocks is fixed at creation (the paper's d_max); all buffers are
 * sized from it (the paper's bucket sizing), and every call brings a new
 * pattern as a COO list of blocks that is re-bucketed on the device.
 *
 * spmm_dynamic_create allocates capacity for max_nnzb blocks of an m x k,
 * block size b operand and n up to any value. opts as for plans (num_panels
 * 0 = one group per panel). */
spmm_status_t spmm_dynamic_create(int64_t m, int64_t k, int32_t b, int64_t max_nnzb,
                                  spmm_dtype_t w, spmm_dtype_t x, spmm_dtype_t y,
                                  const spmm_plan_opts* opts, spmm_dyn_t* out);

/* One dynamic call. nnzb_dev: device int32 holding the number of blocks of
 * this call (read on the device, so the call can be captured in a graph).
 * block_row_dev / block_col_dev: int32 [nnzb], any order, duplicates allowed
 * (summed). values_dev: [nnzb][b][b] of dtype w in the same order as the
 * indices. scales_dev: FP32 [nnzb] for FP8, else NULL. status_dev: device
 * int32 that receives SPMM_OK, SPMM_ERR_CAPACITY (nnzb > max_nnzb or < 0) or
 * SPMM_ERR_BAD_INDEX (an index outside the block grid); on a non-OK status Y
 * is left untouched. The index and value buffers must hold max_nnzb entries'
 * worth of readable memory only up to the nnzb actually used. The first call
 * of a handle for an n class (the power of two at or above n) times the
 * call's variants on its own operands, encoding included, as spmm_run_static
 * does for a plan (it synchronises `stream`; not with SPMM_AUTOTUNE=0 or on a
 * stream under capture, where the rules choose); later calls of that class
 * run the fastest. The variants are the compute kernel's forms after an
 * encoder launch, and, for b = 16 with W in the X type (FP16 or BF16), k a
 * multiple of 16 and max_nnzb up to 2^16 blocks (keys in 64 KiB of LDS),
 * form 5: one launch in which every workgroup (a block row and a column
 * tile) reads the whole COO list, keeps and sorts its row's entries and runs
 * form 4's product on them, writing the call's block-CSR on the way. The
 * rule takes form 5 where it takes form 4 and the workgroups' redundant
 * reads of the list stay under 2^24 entries (SPMM_DYN_FUSED=0/1 forces the
 * choice). Results equal a static plan's of the same pattern bit for bit when
 * both run the same variant (form 5 as form 4). */
spmm_status_t spmm_run_dynamic(spmm_dyn_t h, const int32_t* nnzb_dev, const int32_t* block_row_dev,
                               const int32_t* block_col_dev, const void* values_dev,
                               const float* scales_dev, int64_t n, const void* X, int64_t ldx,
                               void* Y, int64_t ldy, int32_t* status_dev, void* stream);

/* Host copies of the plan the last spmm_run_dynamic built (synchronises the
 * handle's work): row_ptr int32 [mb + 1], col_idx int32 [nnzb], src int32
 * [nnzb] (input index of each CSR entry), panel_ptr int32 [num_panels + 1].
 * *nnzb receives the block count of that call. */
spmm_status_t spmm_dynamic_export(spmm_dyn_t h, int32_t* row_ptr, int32_t* col_idx, int32_t* src,
                                  int32_t* panel_ptr, int64_t* nnzb);

spmm_status_t spmm_dynamic_info(spmm_dyn_t h, int32_t* group_rows, int32_t* num_groups,
                                int32_t* num_panels);

spmm_status_t spmm_dynamic_destroy(spmm_dyn_t h);

/* ------------------------------------------------------- allocation-free dynamic call
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. The same
 * call as spmm_run_dynamic (same kernels, same results bit for bit) without a
 * handle: the shape and capacity come as arguments, and the encoder's buffers
 * (block-CSR of the call, input indices, panels, status) live in a fixed
 * array of SPMM_NOALLOC_SCRATCH_BYTES of device memory that the library
 * holds on every GPU it runs on until the process ends. Nothing is
 * allocated, ever. Limits: b must divide k, and the call must fit the
 * one-workgroup encoder and the array: (mb + 1) + 2 max_nnzb + (panels + 1) + 64
 * int32 words (for example m = k = 4096, b = 16, max_nnzb = 8192 uses about 65 KiB);
 * beyond them the call returns SPMM_ERR_CAPACITY before enqueueing anything.
 * Every call on one GPU uses the same array: calls that overlap on one GPU
 * (different streams, or threads) race and must be ordered by the caller.
 * The values are read in place (not copied), so they must stay valid until
 * the call's work on `stream` completes. Other arguments, errors and the
 * device status word as for spmm_run_dynamic. */
#define SPMM_NOALLOC_SCRATCH_BYTES (256 * 1024)
spmm_status_t spmm_run_dynamic_noalloc(int64_t m, int64_t k, int32_t b, int64_t max_nnzb,
                                       spmm_dtype_t w, spmm_dtype_t x, spmm_dtype_t y,
                                       const int32_t* nnzb_dev, const int32_t* block_row_dev,
                                       const int32_t* block_col_dev, const void* values_dev,
                                       const float* scales_dev, int64_t n, const void* X, int64_t ldx,
                                       void* Y, int64_t ldy, int32_t* status_dev, void* stream);

/* ------------------------------------------------------------------ serving
 * A request loop for a chain of sparse layers whose weights stay resident on
 * the device: y = f_L(... f_1(x)), f_l(v) = act_l((M o W)_l v), where act_l is
 * ReLU when relu_after[l] != 0 and the identity otherwise. The paper's closing
 * motivation is faster inference of large sparse models (Section 6); this loop
 * is built on its static products.
 *
 * A request is n columns (tokens): x_host is [dims[0] x n] and y_host
 * [dims[L] x n], row-major with leading dimension ld_host >= n (elements),
 * host memory the caller keeps valid until the request is reported done.
 * Copies are asynchronous DMA when the buffers are pinned (hipHostMalloc) and
 * ld_host is n rounded up to a multiple of 8 (the device layout); other
 * layouts take a strided copy. Activations live in a device pool of
 * mem_budget_bytes; a request holds two ping-pong buffers of
 * n8 * (largest even-side dim + largest odd-side dim) elements (n8 = n rounded
 * up to a multiple of 8) from admission to completion.
 *
 * CONTINUOUS mode (continuous batching): requests are admitted in arrival
 * order whenever the pool and max_active allow, also while others are in
 * flight; every step advances each admitted request by one layer, all of them
 * in one grouped launch (spmm_group_run, fused ReLU), so requests at different
 * layers share the device. PLAIN mode is the one-call-per-request reference:
 * one request at a time, in arrival order, one spmm_run_static plus one ReLU
 * kernel per layer.
 *
 * A worker thread runs the steps unless opts.manual is set; then the caller
 * drives them with spmm_serve_step. The worker keeps up to two steps enqueued
 * on the device ahead of the one that completes; a manual step completes
 * before it returns. opts.simulate runs the scheduler without
 * any device work (plans may be NULL; dims are required): admission, memory
 * accounting and completion order are those of a real run, outputs are not
 * written. */
typedef enum { SPMM_SERVE_CONTINUOUS = 0, SPMM_SERVE_PLAIN = 1 } spmm_serve_mode_t;

typedef struct {
  int64_t mem_budget_bytes;  /* device activation pool */
  int32_t max_active;        /* requests in flight at most (CONTINUOUS) */
  int32_t mode;              /* spmm_serve_mode_t */
  int32_t manual;            /* nonzero: no worker thread; call spmm_serve_step */
  int32_t simulate;          /* nonzero: scheduler only, no device work */
  int64_t max_tokens;        /* CONTINUOUS: tokens of all admitted requests at most
                                (0 = no limit; a lone request is always admitted) */
} spmm_serve_opts;

typedef struct {
  uint64_t id;
  int64_t n;
  double submit_s;  /* spmm_serve_clock() at submission */
  double admit_s;   /* ... at admission (activation memory granted) */
  double done_s;    /* ... when the output was in y_host */
} spmm_serve_done_t;

typedef struct {
  int64_t steps;           /* grouped steps (CONTINUOUS) or requests run (PLAIN) */
  int64_t requests_done;
  int64_t tokens_done;
  int64_t problems_run;    /* layer products executed */
  int64_t peak_pool_bytes; /* most activation memory held at once */
  int32_t peak_active;     /* most requests in flight at once */
  int32_t pending;         /* submitted, not yet admitted */
  int32_t active;          /* admitted, not yet done */
  int32_t reserved;
  double busy_s;           /* wall time spent inside steps */
} spmm_serve_stats_t;

/* layer_plans: [num_layers] plans with values set (NULL allowed only when
 * simulating); dims: [num_layers + 1] feature sizes, dims[l] = k of layer l
 * and dims[l + 1] = m of layer l (checked against the plans); relu_after:
 * [num_layers] or NULL (no activation). The plans must chain (m of layer l =
 * k of layer l + 1, y dtype of l = x dtype of l + 1) and, in CONTINUOUS mode,
 * satisfy spmm_group_run's conditions. The plans must outlive the server.
 * Errors: INVALID_ARG, UNSUPPORTED, OOM, HIP. */
spmm_status_t spmm_serve_create(const spmm_plan_t* layer_plans, int32_t num_layers, const int64_t* dims,
                                const uint8_t* relu_after, const spmm_serve_opts* opts, spmm_srv_t* out);

/* Queues a request. Returns REJECTED when its activation buffers exceed the
 * whole pool (it could never be admitted), INVALID_ARG for n < 1, ld_host < n
 * or NULL buffers (outside simulation), HIP/... if the server has failed. */
spmm_status_t spmm_serve_submit(spmm_srv_t srv, uint64_t id, int64_t n, const void* x_host, void* y_host,
                                int64_t ld_host);

/* Moves up to max finished requests into out (completion order) and sets
 * *num_done. Never blocks. */
spmm_status_t spmm_serve_poll(spmm_srv_t srv, spmm_serve_done_t* out, int32_t max, int32_t* num_done);

/* Manual mode: one step (admission + one layer for every admitted request in
 * CONTINUOUS mode, one whole request in PLAIN mode), synchronous. *active_out
 * (may be NULL) receives the requests still in flight or pending. */
spmm_status_t spmm_serve_step(spmm_srv_t srv, int32_t* active_out);

/* Blocks until every submitted request is done (worker mode), or runs steps
 * until then (manual mode). Returns the server's failure status if any. */
spmm_status_t spmm_serve_drain(spmm_srv_t srv);

spmm_status_t spmm_serve_stats(spmm_srv_t srv, spmm_serve_stats_t* out);

/* Stops the worker after its current step; requests not done are dropped. */
spmm_status_t spmm_serve_destroy(spmm_srv_t srv);

/* The server's clock: seconds on a monotonic host clock. */
double spmm_serve_clock(void);

#ifdef __cplusplus
}
#endif

#endif /* SPMM_H_ */
