// Host-side handle layouts shared by the C-ABI implementation files
// (runtime.cpp: plans and dynamic handles; group.cpp: grouped launches;
// serve.cpp: the serving loop).
#pragma once

#include <map>
#include <tuple>

#include "common.h"

struct spmm_plan_s {
  int64_t m = 0, k = 0;
  int32_t b = 0, mb = 0, kb = 0;
  int64_t nnzb = 0;
  spmm_dtype_t w = SPMM_F32, x = SPMM_F32, y = SPMM_F32;
  spmm::Geometry geo{};
  spmm::PlanBuffers pb;
  void* values = nullptr;      // block-CSR order, edge blocks zeroed past k
  float* scales = nullptr;     // FP8 block scales, CSR order
  bool has_values = false;
  int device = 0;
  int32_t variant_opt = 0;     // fixed tile variant from the options, 0 = choose
  int32_t tuned[32] = {};      // autotuned variant per n class, 0 = none
  int32_t num_heavy = 0;       // block rows the row-wise kernel splits over four waves
  int32_t* light_rows = nullptr;   // device [mb - num_heavy]: rows of the light units, longest first (skewed plans)
  int32_t* heavy_rows = nullptr;   // device [num_heavy]
  // Long rows cut into pieces (none cut: all zero). Entries [row, first
  // block, end block, slot, c, C, 0, 0]; slots number the cut pieces in row
  // order, the same in both tables.
  int32_t num_pieces = 0;          // pieces of the split rows
  int32_t* pieces = nullptr;       // device [num_pieces][8]
  int32_t num_pieces_all = 0;      // pieces of every row (the every-row split form)
  int32_t* pieces_all = nullptr;   // device [num_pieces_all][8]
  int32_t num_slots = 0;           // cut pieces: partial slots
  int32_t num_cut = 0;             // rows cut into pieces
  bool pieces_spread = false;      // split rows of widely different lengths (plan_pieces)
  int32_t* cut_rows = nullptr;     // device [num_cut][4]: row, first slot, C, 0
  // Piece workspace, grown on a run with more columns than it holds: the
  // partials of num_slots slots for up to piece_ws_n columns.
  float* piece_part = nullptr;
  int64_t piece_ws_n = 0;
  int64_t piece_ws_bytes = 0;
  int32_t* sddmm_tasks = nullptr;  // device [sddmm_num_tasks][2] (16-bit X, b <= 32)
  int32_t sddmm_num_tasks = 0;
  int32_t* sddmm_tiled_tasks = nullptr;  // device [n][4] (b = 16/32): tile row, tile column, first, count
  int32_t* sddmm_tiled_ent = nullptr;    // device [nnzb][2]: CSR index, packed block position in its tile
  int32_t sddmm_tiled_num = 0;
  float* sddmm_dense_ws = nullptr;    // device panel for the dense-GEMM weight gradient, from its first use
  int64_t sddmm_dense_ws_bytes = 0;
  double predicted_speedup = 0.0;  // speedup model's sparse/dense ratio for this plan's shape
  int32_t dense_mode = 0;          // dense dispatch option (0 off, 1 where the model favours dense, 2 always)
  void* dense_w = nullptr;         // dense copy of M o W (m x k, row-major) when the plan keeps one
  int32_t ell_width = 0;           // plans built from blocked-ELL: slots per block row
  int32_t* ell_slot = nullptr;     // device [nnzb]: ELL slot (row * ell_width + slot) of each CSR entry
};

namespace spmm {

// n class of the autotuner: the exponent of the power of two at or above n.
int n_class(int64_t n);
// A tile variant: column tiles of 16 per wave (b >= 16) or columns per lane
// (b < 16) in the low byte, 0 = the rule on n; above it the kernel form: 0 =
// the rule, 1 = the plain kernel, 2 = the other form where the plan has one
// (the software-pipelined row kernel for b = 16/32 with W in the X type and
// no split rows; the LDS-staged kernel for b = 4 with W in the X type), 3 =
// the dense GEMM on the plan's dense copy (plans with dense dispatch), 4 = the
// row kernel with every block row split over a workgroup's four waves (b =
// 16, 16-bit X), 5 = dynamic calls only: form 4 with the encoding in the same
// launch.
constexpr int kFormShift = 8;
inline int32_t variant_ns(int32_t v) { return v & 0xff; }
inline int32_t variant_form(int32_t v) { return v >> kFormShift; }
inline int32_t make_variant(int32_t ns, int32_t form) { return ns | (form << kFormShift); }
bool valid_variant(int32_t b, int32_t v);
// Tile variant for a run of `p` with n columns: fixed option, else the plan's
// tuned value, else the process-wide tuned table, else the rule on n.
int32_t plan_variant(const spmm_plan_s* p, int64_t n);
// Whether a run of n columns at tile width ns uses the plan's pieces of long
// rows (split_all: in the every-row split form).
bool plan_pieces(const spmm_plan_s* p, int64_t n, int32_t ns, bool split_all);
// Whether the plan runs on the row-wise MFMA kernel (b = 16/32/64, 16-bit X).
bool plan_uses_row_kernel(const spmm_plan_s* p);
// Whether a run with n columns, tile width ns and this variant splits every
// block row (form 4, else the rule split_all_preferred; SPMM_SPLIT_ALL forces).
bool plan_split_all(const spmm_plan_s* p, int64_t n, int32_t ns, int32_t variant);
// Enqueues Y = (M o W) X for a validated plan (no argument checks).
spmm_status_t run_plan(const spmm_plan_s* p, int64_t n, const void* X, int64_t ldx, void* Y, int64_t ldy,
                       int32_t variant, bool relu, hipStream_t stream);
// The compute kernel of a dynamic call (a.plan, a.n, dtypes, W, status set).
spmm_status_t run_dynamic_kernel(RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx, hipStream_t s,
                                 int32_t variant = 0);
spmm_status_t check_dense(const void* p, int64_t ld, int64_t n, int elem, const char* name);
spmm_status_t check_device(int device);
int32_t default_ns(int64_t n);

// Dense dispatch (dense.hip): whether a plan with these dtypes can keep a
// dense copy; (re)builds the copy from the plan's CSR values on `s`; runs
// Y = Wd X with a library GEMM on `s`.
bool dense_dispatch_eligible(spmm_dtype_t w, spmm_dtype_t x, spmm_dtype_t y);
spmm_status_t build_dense_copy(spmm_plan_s* p, hipStream_t s);
spmm_status_t run_dense(const spmm_plan_s* p, int64_t n, const void* X, int64_t ldx, void* Y, int64_t ldy,
                        hipStream_t s);
// Weight gradient by a dense GEMM: dY X^T (FP32, library GEMM) in row panels
// of sddmm_dense_panel_rows rows in ws (panel rows x k floats), the mask's
// blocks gathered into G in CSR order.
int64_t sddmm_dense_panel_rows(const spmm_plan_s* p);
spmm_status_t sddmm_dense(const spmm_plan_s* p, int64_t n, const void* dY, int64_t lddy, const void* X, int64_t ldx,
                          float* G, float* ws, hipStream_t s);

// Autotuner table persisted as JSON (tune_cache.cpp). Key: (b, w, x, y,
// density class, n class, dense copy kept: its candidates include the dense
// GEMM). load fills `table` from `path` when the file was
// written for this device and HIP runtime (else leaves it unchanged); save
// writes the whole table (a temporary file renamed over `path`). Both return
// false on an unreadable or unwritable file and never fail a product.
using TuneKey = std::tuple<int, int, int, int, int, int, int>;
bool tune_cache_load(const char* path, std::map<TuneKey, int32_t>& table);
bool tune_cache_save(const char* path, const std::map<TuneKey, int32_t>& table);

}  // namespace spmm
