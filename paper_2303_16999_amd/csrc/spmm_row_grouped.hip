// Grouped launch of the row-wise kernel: one launch runs the work units of many
// problems listed in a table, passed in the kernel arguments (up to 32
// problems) or in device memory.
#include <algorithm>

#include "spmm_row.h"

namespace spmm {
namespace row {

constexpr int kInlineProblems = 28;

// Problem table passed in the kernel arguments (at most kInlineProblems
// problems, 4 KB): no copy precedes the launch.
struct GroupArgs {
  int32_t count, total;
  int32_t pad[2];
  RowProblem probs[kInlineProblems];
};

// One workgroup per work unit of the group; a unit is (problem, group of 4
// block rows, column tile of 16*ns). Each problem owns a range of workgroups
// starting at a multiple of 8, so the dispatcher's round robin spreads every
// problem evenly over the 8 XCDs (as a launch of its own would be); inside
// the range the units are numbered XCD-contiguously. The problem of a
// workgroup is the last one whose range starts at or before it.
template <typename XT, typename WT, typename YT, int B, bool SPLIT>
__device__ __forceinline__ void group_unit(const RowProblem* __restrict__ probs, int32_t count, int32_t total,
                                           float4_t* red) {
  const int lane = threadIdx.x & 63;
  const int wave = SPLIT ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : (int)(threadIdx.x >> 6);
  const int32_t wg = blockIdx.x;
  int32_t lo = 0, hi = count - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (uniform(probs[mid].unit_begin) <= wg) lo = mid;
    else hi = mid - 1;
  }
  const RowProblem p = probs[lo];  // by value: the fields live in scalar registers
  const int32_t nu = uniform(p.num_units);
  const int32_t w = wg - uniform(p.unit_begin);
  if (w >= nu) return;  // padding up to the next multiple of 8
  const int32_t local = xcd_unit(w, nu);
  const int32_t ns = uniform(p.ns);
  if (ns == 8) row_unit<XT, WT, YT, B, 8, SPLIT>(p, local, lane, wave, red);
  else if (ns == 4) row_unit<XT, WT, YT, B, 4, SPLIT>(p, local, lane, wave, red);
  else row_unit<XT, WT, YT, B, 2, SPLIT>(p, local, lane, wave, red);
}

// Persistent form: a grid of a few workgroups per CU (a multiple of 8, so
// that every XCD runs the same number) walks the work units itself. The units
// are split into 8 queues: queue x lists, problem after problem, the
// contiguous range of each problem's units that the launch-per-unit form
// gives XCD x, so every XCD keeps working on a few column tiles at a time, as
// in that form. Workgroup w serves queue w % 8 (the dispatcher's round robin
// over the XCDs; any other placement changes locality, not results) and takes
// its entries w / 8, w / 8 + G / 8, ... for a grid of G: a static schedule,
// with no counters to keep between launches.
template <typename XT, typename WT, typename YT, int B, bool SPLIT>
__device__ __forceinline__ void group_persist(const RowProblem* __restrict__ probs, int32_t count, float4_t* red) {
  const int lane = threadIdx.x & 63;
  const int wave = SPLIT ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : (int)(threadIdx.x >> 6);
  const int32_t x = blockIdx.x & 7;
  const int32_t stride = gridDim.x >> 3;
  int32_t i = blockIdx.x >> 3;  // entry of queue x
  int32_t base = 0;             // entry where problem pi's share starts
  for (int32_t pi = 0; pi < count; ++pi) {
    // XCD x's share of a problem of nu = 8 q + r units: units x q + min(x, r)
    // onward, q + (x < r) of them
    const int32_t nu = uniform(probs[pi].num_units);
    const int32_t q = nu >> 3, r = nu & 7;
    const int32_t len = q + (x < r ? 1 : 0);
    if (i - base >= len) {
      base += len;
      continue;
    }
    const RowProblem p = probs[pi];
    const int32_t ns = uniform(p.ns);
    const int32_t first = x * q + min(x, r) - base;
    for (; i - base < len; i += stride) {
      if (ns == 8) row_unit<XT, WT, YT, B, 8, SPLIT>(p, first + i, lane, wave, red);
      else if (ns == 4) row_unit<XT, WT, YT, B, 4, SPLIT>(p, first + i, lane, wave, red);
      else row_unit<XT, WT, YT, B, 2, SPLIT>(p, first + i, lane, wave, red);
      if (SPLIT) __syncthreads();  // a split unit's LDS is read by all before the next unit writes it
    }
    base += len;
  }
}

template <typename XT, typename WT, typename YT, int B, bool SPLIT>
__global__ __launch_bounds__(256, B == 16 ? 4 : 3) void k_spmm_row_grouped_persist(GroupArgs args) {
  extern __shared__ float4_t grp_red[];
  group_persist<XT, WT, YT, B, SPLIT>(args.probs, args.count, SPLIT ? grp_red : nullptr);
}

template <typename XT, typename WT, typename YT, int B, bool SPLIT>
__global__ __launch_bounds__(256, B == 16 ? 4 : 3) void k_spmm_row_grouped_persist_table(
    const RowProblem* __restrict__ probs, int32_t count) {
  extern __shared__ float4_t grp_red[];
  group_persist<XT, WT, YT, B, SPLIT>(probs, count, SPLIT ? grp_red : nullptr);
}

// Table in device memory (any number of problems). SPLIT: some problem has
// split rows (b = 16 only).
template <typename XT, typename WT, typename YT, int B, bool SPLIT>
__global__ __launch_bounds__(256, B == 16 ? 4 : 3) void k_spmm_row_grouped(const RowProblem* __restrict__ probs,
                                                                          int32_t count, int32_t total) {
  extern __shared__ float4_t grp_red[];
  group_unit<XT, WT, YT, B, SPLIT>(probs, count, total, SPLIT ? grp_red : nullptr);
}

// Table in the kernel arguments.
template <typename XT, typename WT, typename YT, int B, bool SPLIT>
__global__ __launch_bounds__(256, B == 16 ? 4 : 3) void k_spmm_row_grouped_args(GroupArgs args) {
  extern __shared__ float4_t grp_red[];
  group_unit<XT, WT, YT, B, SPLIT>(args.probs, args.count, args.total, SPLIT ? grp_red : nullptr);
}

}  // namespace row
}  // namespace spmm

namespace spmm {

namespace {
template <typename XT, typename YT>
const void* args_kernel_b(int32_t b, bool split) {
  if (b == 16 && split) return reinterpret_cast<const void*>(&row::k_spmm_row_grouped_args<XT, XT, YT, 16, true>);
  if (b == 16) return reinterpret_cast<const void*>(&row::k_spmm_row_grouped_args<XT, XT, YT, 16, false>);
  return reinterpret_cast<const void*>(&row::k_spmm_row_grouped_args<XT, XT, YT, 32, false>);
}

template <typename XT, typename YT>
void table_launch_b(int32_t b, bool split, const row::RowProblem* probs, int32_t count, int32_t total, unsigned lds,
                    hipStream_t s) {
  if (b == 16 && split)
    hipLaunchKernelGGL((row::k_spmm_row_grouped<XT, XT, YT, 16, true>), dim3((unsigned)total), dim3(256), lds, s, probs,
                       count, total);
  else if (b == 16)
    hipLaunchKernelGGL((row::k_spmm_row_grouped<XT, XT, YT, 16, false>), dim3((unsigned)total), dim3(256), 0, s,
                       probs, count, total);
  else
    hipLaunchKernelGGL((row::k_spmm_row_grouped<XT, XT, YT, 32, false>), dim3((unsigned)total), dim3(256), 0, s,
                       probs, count, total);
}
}  // namespace

namespace {
template <typename XT, typename YT>
spmm_status_t persist_launch_b(int32_t b, bool split, const void* args, const row::RowProblem* probs, int32_t count,
                               int32_t grid, unsigned lds, hipStream_t s) {
  if (args) {
    const row::GroupArgs& ga = *(const row::GroupArgs*)args;
    if (b == 16 && split)
      hipLaunchKernelGGL((row::k_spmm_row_grouped_persist<XT, XT, YT, 16, true>), dim3((unsigned)grid), dim3(256), lds,
                         s, ga);
    else if (b == 16)
      hipLaunchKernelGGL((row::k_spmm_row_grouped_persist<XT, XT, YT, 16, false>), dim3((unsigned)grid), dim3(256), 0,
                         s, ga);
    else
      hipLaunchKernelGGL((row::k_spmm_row_grouped_persist<XT, XT, YT, 32, false>), dim3((unsigned)grid), dim3(256), 0,
                         s, ga);
  } else {
    if (b == 16 && split)
      hipLaunchKernelGGL((row::k_spmm_row_grouped_persist_table<XT, XT, YT, 16, true>), dim3((unsigned)grid), dim3(256),
                         lds, s, probs, count);
    else if (b == 16)
      hipLaunchKernelGGL((row::k_spmm_row_grouped_persist_table<XT, XT, YT, 16, false>), dim3((unsigned)grid),
                         dim3(256), 0, s, probs, count);
    else
      hipLaunchKernelGGL((row::k_spmm_row_grouped_persist_table<XT, XT, YT, 32, false>), dim3((unsigned)grid),
                         dim3(256), 0, s, probs, count);
  }
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}
}  // namespace

// Workgroups of a persistent grouped launch: about `per_cu` per CU (the
// occupancy of the row-wise kernel), a multiple of 8, and never more than the
// launch-per-unit form would start.
int32_t group_persist_grid(int32_t total_units, int per_cu) {
  const int64_t cap = (int64_t)device_cu_count() * per_cu;
  const int64_t g = std::min<int64_t>(cap, (int64_t)total_units);
  return (int32_t)std::max<int64_t>(8, (g + 7) & ~(int64_t)7);
}

spmm_status_t launch_spmm_row_grouped_persist(spmm_dtype_t xt, spmm_dtype_t yt, int32_t b, const void* args,
                                              const void* probs_dev, int32_t count, int32_t grid, unsigned lds,
                                              hipStream_t s) {
  using bf = __bf16;
  if (b != 16 && b != 32) return fail(SPMM_ERR_UNSUPPORTED, "grouped launch handles block sizes 16 and 32");
  const row::RowProblem* pr = (const row::RowProblem*)probs_dev;
  const bool split = lds > 0;
  if (xt == SPMM_F16) {
    if (yt == SPMM_F32) return persist_launch_b<_Float16, float>(b, split, args, pr, count, grid, lds, s);
    return persist_launch_b<_Float16, _Float16>(b, split, args, pr, count, grid, lds, s);
  }
  if (xt == SPMM_BF16) {
    if (yt == SPMM_F32) return persist_launch_b<bf, float>(b, split, args, pr, count, grid, lds, s);
    return persist_launch_b<bf, bf>(b, split, args, pr, count, grid, lds, s);
  }
  return fail(SPMM_ERR_UNSUPPORTED, "grouped launch needs 16-bit X");
}

int32_t group_inline_max() { return row::kInlineProblems; }
size_t group_args_bytes() { return sizeof(row::GroupArgs); }
size_t row_problem_size() { return sizeof(row::RowProblem); }

void group_args_header(void* args, int32_t count, int32_t total) {
  row::GroupArgs* g = (row::GroupArgs*)args;
  g->count = count;
  g->total = total;
  g->pad[0] = g->pad[1] = 0;
}

void* group_args_problem(void* args, int32_t i) { return &((row::GroupArgs*)args)->probs[i]; }

// Fills one problem descriptor (host side; layout shared with the kernels).
void fill_row_problem(void* dst, const RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx,
                      int32_t unit_begin, int32_t num_units) {
  row::RowProblem p = row::row_problem(a, row_ptr, col_idx);
  p.unit_begin = unit_begin;
  p.num_units = num_units;
  *(row::RowProblem*)dst = p;
}

// Kernel of the argument-table form for a dtype class (16-bit W = X), or
// nullptr. split: some problem of the group has split rows (b = 16).
const void* row_grouped_args_kernel(spmm_dtype_t xt, spmm_dtype_t yt, int32_t b, bool split) {
  using bf = __bf16;
  if (b != 16 && b != 32) return nullptr;
  if (xt == SPMM_F16)
    return yt == SPMM_F32 ? args_kernel_b<_Float16, float>(b, split) : args_kernel_b<_Float16, _Float16>(b, split);
  if (xt == SPMM_BF16) return yt == SPMM_F32 ? args_kernel_b<bf, float>(b, split) : args_kernel_b<bf, bf>(b, split);
  return nullptr;
}

spmm_status_t launch_spmm_row_grouped_args(spmm_dtype_t xt, spmm_dtype_t yt, int32_t b, const void* args, int32_t total,
                                           unsigned lds, hipStream_t s) {
  const void* fn = row_grouped_args_kernel(xt, yt, b, lds > 0);
  if (!fn) return fail(SPMM_ERR_UNSUPPORTED, "grouped launch needs 16-bit X and b = 16 or 32");
  void* params[1] = {const_cast<void*>(args)};
  SPMM_HIP(hipLaunchKernel(fn, dim3((unsigned)total), dim3(256), params, lds, s));
  return SPMM_OK;
}

// LDS of a grouped launch whose problems include split rows.
unsigned group_split_lds(int32_t b) { return (unsigned)row::split_lds_bytes(b, 8); }

int64_t group_problem_units(int32_t num_light, int64_t n, int32_t ns, int32_t num_heavy, bool inter) {
  return row::problem_units(num_light, n, ns, num_heavy, inter);
}

spmm_status_t launch_spmm_row_grouped(spmm_dtype_t xt, spmm_dtype_t yt, int32_t b, const void* probs_dev,
                                      int32_t count, int32_t total, unsigned lds, hipStream_t s) {
  using bf = __bf16;
  const row::RowProblem* pr = (const row::RowProblem*)probs_dev;
  if (b != 16 && b != 32) return fail(SPMM_ERR_UNSUPPORTED, "grouped launch handles block sizes 16 and 32");
  if (xt == SPMM_F16) {
    if (yt == SPMM_F32) table_launch_b<_Float16, float>(b, lds > 0, pr, count, total, lds, s);
    else table_launch_b<_Float16, _Float16>(b, lds > 0, pr, count, total, lds, s);
  } else if (xt == SPMM_BF16) {
    if (yt == SPMM_F32) table_launch_b<bf, float>(b, lds > 0, pr, count, total, lds, s);
    else table_launch_b<bf, bf>(b, lds > 0, pr, count, total, lds, s);
  } else {
    return fail(SPMM_ERR_UNSUPPORTED, "grouped launch needs 16-bit X");
  }
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

spmm_status_t launch_group_fixup(const RunArgs& a, int ns, hipStream_t stream) {
  if (!a.part || a.num_cut == 0 || a.n == 0) return SPMM_OK;
  const row::RowProblem pr = row::row_problem(a, nullptr, nullptr);
  switch (a.yt) {
    case SPMM_F16: return row::launch_piece_fixup<_Float16>(pr, a.cut_rows, a.num_cut, ns, stream);
    case SPMM_BF16: return row::launch_piece_fixup<__bf16>(pr, a.cut_rows, a.num_cut, ns, stream);
    case SPMM_F32: return row::launch_piece_fixup<float>(pr, a.cut_rows, a.num_cut, ns, stream);
    default: return fail(SPMM_ERR_UNSUPPORTED, "output dtype");
  }
}

}  // namespace spmm
