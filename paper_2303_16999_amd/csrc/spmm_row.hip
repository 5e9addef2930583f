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
  return fail(SPMM_ERR_UNSUPPORTED, "row-wise kernel handles block sizes 16 and 32");
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

namespace spmm {

// Grouped persistent launch of the row-wise kernel (16-bit W and X).
template <typename XT, typename YT>
static spmm_status_t grouped_b(int32_t b, const void* probs, const int32_t* header, int32_t grid, hipStream_t s) {
  const row::RowProblem* pr = (const row::RowProblem*)probs;
  if (b == 16) return row::launch_row_grouped<XT, XT, YT, 16>(pr, header, grid, s);
  if (b == 32) return row::launch_row_grouped<XT, XT, YT, 32>(pr, header, grid, s);
  return fail(SPMM_ERR_UNSUPPORTED, "grouped launch handles block sizes 16 and 32");
}

spmm_status_t launch_spmm_row_grouped(spmm_dtype_t xt, spmm_dtype_t yt, int32_t b, const void* probs_dev,
                                      const int32_t* header_dev, int32_t grid, hipStream_t s) {
  using bf = __bf16;
  if (xt == SPMM_F16) return yt == SPMM_F32 ? grouped_b<_Float16, float>(b, probs_dev, header_dev, grid, s)
                                            : grouped_b<_Float16, _Float16>(b, probs_dev, header_dev, grid, s);
  if (xt == SPMM_BF16) return yt == SPMM_F32 ? grouped_b<bf, float>(b, probs_dev, header_dev, grid, s)
                                             : grouped_b<bf, bf>(b, probs_dev, header_dev, grid, s);
  return fail(SPMM_ERR_UNSUPPORTED, "grouped launch needs 16-bit X");
}

size_t row_problem_size() { return sizeof(row::RowProblem); }

template <typename XT, typename YT, int B>
static int32_t occupancy() {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&row::k_spmm_row_grouped<XT, XT, YT, B>),
                                                   256, 0) != hipSuccess)
    per_cu = 1;
  return per_cu > 0 ? per_cu : 1;
}

// Workgroups of a persistent grouped launch: every slot the occupancy allows on every CU.
int32_t row_grouped_grid(spmm_dtype_t xt, spmm_dtype_t yt, int32_t b) {
  using bf = __bf16;
  int32_t per_cu;
  if (xt == SPMM_F16) per_cu = b == 16 ? (yt == SPMM_F32 ? occupancy<_Float16, float, 16>() : occupancy<_Float16, _Float16, 16>())
                                       : (yt == SPMM_F32 ? occupancy<_Float16, float, 32>() : occupancy<_Float16, _Float16, 32>());
  else per_cu = b == 16 ? (yt == SPMM_F32 ? occupancy<bf, float, 16>() : occupancy<bf, bf, 16>())
                        : (yt == SPMM_F32 ? occupancy<bf, float, 32>() : occupancy<bf, bf, 32>());
  return per_cu * device_cu_count();
}

// Fills one descriptor of the grouped table (host side; layout shared with the kernel).
void fill_row_problem(void* dst, const RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx,
                      int32_t unit_begin) {
  row::RowProblem p = row::row_problem(a, row_ptr, col_idx);
  p.unit_begin = unit_begin;
  *(row::RowProblem*)dst = p;
}

}  // namespace spmm
