// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/spmm.h"

namespace spmm {

// ------------------------------------------------------------------ errors
// Records a thread-local message and returns the status, so call sites read
// `return fail(SPMM_ERR_INVALID_ARG, "...")`.
spmm_status_t fail(spmm_status_t st, const std::string& msg);
spmm_status_t fail_hip(hipError_t e, const char* what);
void clear_error();

#define SPMM_HIP(call)                                    \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return ::spmm::fail_hip(e_, #call); \
  } while (0)

// ------------------------------------------------------------------ sizes
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
int dtype_bytes(spmm_dtype_t t);
bool dtype_triple_supported(spmm_dtype_t w, spmm_dtype_t x, spmm_dtype_t y);

// ------------------------------------------------------------------ the kernel plan
// Layout consumed by the compute kernels (static plans and dynamic calls build
// the same): block-CSR (row_ptr, col_idx; columns ascending inside a row),
// row groups of group_rows consecutive block rows, the cost-balanced panels of
// the groups, and the in-group column-major order (order[q] is the CSR
// position of the q-th block when each group lists its blocks by (block
// column, block row); groups follow each other).
struct KernelPlan {
  int32_t m, k, b;
  int32_t mb, kb;
  int32_t group_rows;   // block rows per group
  int32_t num_groups;
  int32_t num_panels;
  const int32_t* panel_ptr;  // [num_panels + 1], group indices
  const int32_t* order;      // [nnz] (static plans; nullptr for dynamic calls)
};

// Device buffers that back a KernelPlan.
struct PlanBuffers {
  int32_t* panel_ptr = nullptr;
  int32_t* row_ptr = nullptr;
  int32_t* col_idx = nullptr;   // CSR columns
  int32_t* order = nullptr;     // static: in-group column-major order of CSR positions
  int32_t* csr_src = nullptr;   // dynamic: input index of each CSR entry
  int32_t* tmp_col = nullptr;   // dynamic: [max_nnz] scratch of the multi-kernel encoder's row sort
  int32_t* tmp_src = nullptr;
  int32_t* scratch = nullptr;   // counts / scan partials
  int64_t* cost_prefix = nullptr;
  int64_t scratch_ints = 0;
  int32_t* hist = nullptr;      // dynamic: per-workgroup block-row histograms [hist_wgs][mb]
  int32_t hist_wgs = 0;         // workgroups of the histogram encode (0: global-atomic encode)
};
// Workgroups of the dynamic histogram encode for a capacity and block-row
// count (0 where its LDS histogram of mb rows does not fit).
int32_t dyn_hist_wgs(int64_t max_nnz, int32_t mb);

struct Geometry {
  int32_t group_rows, num_groups, num_panels;
};

// Chooses group_rows for a shape. n_hint steers the row-group size so that
// groups x n-tiles fills the chip.
Geometry choose_geometry(int64_t m, int64_t k, int32_t b, int64_t nnz_hint, int64_t n_hint,
                         const spmm_plan_opts* opts, int num_cus, spmm_dtype_t x);

// ------------------------------------------------------------------ plan building kernels
// All of these enqueue on `stream` and do not synchronise.
// Static: block mask -> block-CSR, group costs, panels and the in-group order.
spmm_status_t build_static_plan(const uint8_t* mask_dev, int32_t mb, int32_t kb, const Geometry& geo,
                                PlanBuffers& pb, hipStream_t stream);
// Dynamic, block-CSR form: validate, bucket by block row, sort rows by (column,
// input index), gather values into CSR order, panels from the row groups;
// then the caller's status word and (when nnz_last is not NULL) the entry count.
spmm_status_t build_dynamic_csr(const int32_t* nnz_dev, const int32_t* rows, const int32_t* cols, int32_t max_nnz,
                                int32_t mb, int32_t kb, int32_t b, int32_t k, const Geometry& geo, PlanBuffers& pb,
                                const void* vals, void* vals_out, int elem_bytes, const float* scales,
                                float* scales_out, int32_t* status, int32_t* status_out, int32_t* nnz_last,
                                hipStream_t stream);
// The same encode in one workgroup with the entries in LDS (block-CSR, sources
// and panels only; the values stay where the caller put them and the kernels
// read them through csr_src). Applies when dynamic_small_fits().
bool dynamic_small_fits(int32_t max_nnz, int32_t mb, int32_t kb, int32_t num_groups);
// Row-range encoder: one launch, one workgroup per range of block rows, each
// reading the whole COO list; block-CSR, input indices, status and entry count
// as build_dynamic_csr_small, without panels (dyn_panels derives them from
// row_ptr). Applies when dynamic_rows_fits().
bool dynamic_rows_fits(int32_t max_nnz, int32_t mb, int32_t kb);
spmm_status_t build_dynamic_csr_rows(const int32_t* nnz_dev, const int32_t* rows, const int32_t* cols,
                                     int32_t max_nnz, int32_t mb, int32_t kb, PlanBuffers& pb, int32_t* status,
                                     int32_t* status_out, int32_t* nnz_last, hipStream_t s);
spmm_status_t dyn_panels(const Geometry& geo, int32_t mb, PlanBuffers& pb, const int32_t* status, hipStream_t s);
spmm_status_t build_dynamic_csr_small(const int32_t* nnz_dev, const int32_t* rows, const int32_t* cols,
                                      int32_t max_nnz, int32_t mb, int32_t kb, const Geometry& geo, PlanBuffers& pb,
                                      int32_t* status, int32_t* status_out, int32_t* nnz_last, hipStream_t stream);
// Copy values given in block-CSR order, zeroing the out-of-range part of edge blocks.
spmm_status_t copy_values_csr(const int32_t* col_idx, int64_t nnz, int32_t b, int32_t k, const void* src, void* dst,
                              int elem_bytes, const float* ssrc, float* sdst, hipStream_t stream);

// ------------------------------------------------------------------ compute
struct RunArgs {
  KernelPlan plan;
  const void* W;          // values in block-CSR order (or indexed by w_index)
  const float* scales;    // FP8 block scales (same indexing as W), else nullptr
  const void* X;
  void* Y;
  int64_t ldx, ldy;
  int32_t n;
  spmm_dtype_t wt, xt, yt;
  const int32_t* status;  // skip everything when *status != 0 (dynamic), else nullptr
  int64_t nnz;            // entries in W (capacity for dynamic calls)
  bool relu = false;      // max(0, y) before the output cast
  const int32_t* w_index = nullptr;  // values (and scales) of entry q at w_index[q], else q
  int32_t num_heavy = 0;             // row-wise kernel: split rows (or pieces, with part set)
  const int32_t* light_rows = nullptr;  // [num_light] rows of the light units, in order (nullptr: all rows)
  int32_t num_light = 0;
  const int32_t* heavy_rows = nullptr;  // [num_heavy] split rows, or [num_heavy][8] pieces with part set
  float* part = nullptr;     // piece partials (pieces of long rows), else nullptr
  const int32_t* cut_rows = nullptr;  // [num_cut][4] the rows cut into pieces: row, first slot, C, 0
  int32_t num_cut = 0;
  int32_t ns = 8;         // row-wise kernel: column tiles of 16 per wave (2, 4 or 8)
  bool split_all = false;  // row-wise kernel, b = 16: split every block row (heavy_* unused unless part
                           // is set: then heavy_rows lists the pieces of every row)
};
// Row-wise kernel (16-bit X, b = 16 or 32): W and scales in block-CSR order.
spmm_status_t launch_spmm_row(const RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx, hipStream_t stream);
// Row-wise kernel with a software-pipelined block loop, for launches of at
// most two workgroups per CU (b = 16 or 32, W in the X type; no split rows).
// The same results as launch_spmm_row, bit for bit.
bool row_pp_preferred(int32_t b, int32_t mb, int64_t n, int32_t ns, int64_t nnz, int num_cus);
// Whether the rule splits every block row over a workgroup's four waves (b =
// 16, 16-bit X): launches too small to fill the chip with one wave per row,
// rows long enough to share. SPMM_SPLIT_ALL=0/1 forces the choice.
bool split_all_preferred(int32_t b, int32_t mb, int64_t n, int32_t ns, int64_t nnz, int num_cus);
spmm_status_t launch_spmm_row_pp(const RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx,
                                 hipStream_t stream);
// Row-wise FP32 kernel (FP32 W, X, Y; b = 16 or 32): W in block-CSR order.
spmm_status_t launch_spmm_row_f32(const RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx, hipStream_t stream);
// Grouped row-wise launches (16-bit W and X, b = 16/32): one workgroup per
// work unit of all problems. The table of problem descriptors is either in
// the kernel arguments (at most group_inline_max() problems; built with
// group_args_header / group_args_problem / fill_row_problem) or in device memory.
int32_t group_inline_max();
size_t group_args_bytes();
size_t row_problem_size();
void group_args_header(void* args, int32_t count, int32_t total);
void* group_args_problem(void* args, int32_t i);
void fill_row_problem(void* dst, const RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx,
                      int32_t unit_begin, int32_t num_units);
const void* row_grouped_args_kernel(spmm_dtype_t xt, spmm_dtype_t yt, int32_t b, bool split);
spmm_status_t launch_spmm_row_grouped_args(spmm_dtype_t xt, spmm_dtype_t yt, int32_t b, const void* args,
                                           int32_t total, unsigned lds, hipStream_t stream);
spmm_status_t launch_spmm_row_grouped(spmm_dtype_t xt, spmm_dtype_t yt, int32_t b, const void* probs_dev,
                                      int32_t count, int32_t total, unsigned lds, hipStream_t stream);
// Persistent grouped launch: `grid` workgroups (group_persist_grid, a
// multiple of 8) walk the units of the table (args: the argument form, else
// probs_dev in device memory) on a static per-XCD schedule.
int32_t group_persist_grid(int32_t total_units, int per_cu);
spmm_status_t launch_spmm_row_grouped_persist(spmm_dtype_t xt, spmm_dtype_t yt, int32_t b, const void* args,
                                              const void* probs_dev, int32_t count, int32_t grid, unsigned lds,
                                              hipStream_t stream);
// LDS bytes of a grouped launch with split rows; work units of one problem.
unsigned group_split_lds(int32_t b);
int64_t group_problem_units(int32_t num_light, int64_t n, int32_t ns, int32_t num_heavy, bool inter);
// One-launch dynamic call (b = 16, W in the X type, capacity up to 2^16 blocks
// within the LDS of a workgroup): encode and multiply together, the every-row
// split form's result; writes the call's block-CSR, status and count as the
// encoders do.
bool dynamic_fused_eligible(int32_t b, spmm_dtype_t w, spmm_dtype_t x, spmm_dtype_t y, int64_t k, int32_t mb,
                            int32_t kb, int64_t max_nnz);
bool dynamic_fused_preferred(int32_t mb, int64_t n, int64_t max_nnz);
int32_t dynamic_fused_ns(int64_t n);
spmm_status_t launch_dynamic_fused(const RunArgs& a, const int32_t* nnz_dev, const int32_t* rows, const int32_t* cols,
                                   int32_t max_nnz, int32_t kb, int32_t* row_ptr, int32_t* col_idx, int32_t* src,
                                   int32_t* status, int32_t* status_out, int32_t* nnz_last, hipStream_t s);
// The fixup launch of a problem's cut rows after its pieces ran (grouped
// launches; a single launch issues its own).
spmm_status_t launch_group_fixup(const RunArgs& a, int ns, hipStream_t stream);
// SDDMM (b <= 32, FP16/BF16 dY and X): G[e] = dY[rows of r] X[rows of c]^T
// for the tasks of a plan (block row, first entry, up to sddmm_task_blocks(b)
// blocks each), FP32 output in CSR order.
int32_t sddmm_task_blocks(int32_t b);
// Tiled SDDMM (b = 16/32): tasks of up to sddmm_tiled_task_blocks(b) blocks of
// one tile of sddmm_tiled_tile_blocks(b) x sddmm_tiled_tile_blocks(b) blocks;
// tasks [num_tasks][4] (tile row, tile column, first entry, count), entries
// [nnz][2] (CSR index, block row in tile << 16 | block column in tile).
int32_t sddmm_tiled_tile_blocks(int32_t b);
int32_t sddmm_tiled_task_blocks(int32_t b);
spmm_status_t launch_sddmm_tiled(spmm_dtype_t t, int32_t b, const int32_t* tasks, const int32_t* ent,
                                 int32_t num_tasks, int64_t m, int64_t k, int64_t n, const void* dY, int64_t lddy,
                                 const void* X, int64_t ldx, float* G, hipStream_t s);
spmm_status_t launch_sddmm(spmm_dtype_t t, int32_t b, const int32_t* row_ptr, const int32_t* col_idx,
                           const int32_t* tasks, int32_t num_tasks, int64_t m, int64_t k, int64_t n, const void* dY,
                           int64_t lddy, const void* X, int64_t ldx, float* G, hipStream_t stream);
// Small-block kernels with X staged in LDS for a panel of block rows (b = 1,
// 4 or 8, 16-bit W and X of one type): rows per wave (8, 4 or 2) from
// small_lds_rows_per_wave; small_lds_preferred says whether one runs instead
// of the kernel below (by block size, dtypes, density and n).
bool small_lds_preferred(int32_t b, spmm_dtype_t w, spmm_dtype_t x, int64_t nnz, int64_t mb, int64_t kb, int64_t n);
// Whether an LDS-staged kernel handles the plan at all (b = 1, 4 or 8, W in
// the 16-bit X type).
bool small_lds_eligible(int32_t b, spmm_dtype_t w, spmm_dtype_t x);
int32_t small_lds_rows_per_wave(int32_t b, int32_t mb, int64_t n, int num_cus);
spmm_status_t launch_spmm_small_lds(const RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx, int32_t rw,
                                    hipStream_t stream);
// Small-block kernel (b = 1, 4, 8, every dtype triple): W and scales in block-CSR order.
spmm_status_t launch_spmm_small(const RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx, hipStream_t stream);


int device_cu_count();

}  // namespace spmm
