// Instantiations of the row-wise SpMM kernel.
#include "spmm_row.h"

namespace spmm {

template <typename XT, typename WT>
static spmm_status_t row_y(const RunArgs& a, const int32_t* rp, const int32_t* ci, hipStream_t s) {
  if (a.plan.b == 16) {
    if (a.yt == SPMM_F32) return row::launch_row<XT, WT, float, 16>(a, rp, ci, s);
    return row::launch_row<XT, WT, XT, 16>(a, rp, ci, s);
  }
  if (a.plan.b == 32) {
    if (a.yt == SPMM_F32) return row::launch_row<XT, WT, float, 32>(a, rp, ci, s);
    return row::launch_row<XT, WT, XT, 32>(a, rp, ci, s);
  }
  if (a.plan.b == 64) {
    if (a.yt == SPMM_F32) return row::launch_row<XT, WT, float, 64>(a, rp, ci, s);
    return row::launch_row<XT, WT, XT, 64>(a, rp, ci, s);
  }
  return fail(SPMM_ERR_UNSUPPORTED, "row-wise kernel handles block sizes 16, 32 and 64");
}

spmm_status_t launch_spmm_row(const RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx, hipStream_t s) {
  using bf = __bf16;
  if (a.wt == SPMM_FP8_E4M3) {
    if (a.xt == SPMM_F16) return row_y<_Float16, row::Fp8>(a, row_ptr, col_idx, s);
    return row_y<bf, row::Fp8>(a, row_ptr, col_idx, s);
  }
  if (a.xt == SPMM_F16) return row_y<_Float16, _Float16>(a, row_ptr, col_idx, s);
  return row_y<bf, bf>(a, row_ptr, col_idx, s);
}

}  // namespace spmm
