// Dynamic-mode SpMM that allocates nothing: spmm_run_dynamic_noalloc.
//
// The same encode and compute kernels as spmm_run_dynamic on its
// one-workgroup path (the block-CSR of the call, its input indices, panels
// and status word built by one workgroup; values read where the caller put
// them), with the device buffers those kernels need taken from a fixed array
// in device memory instead of a handle's allocations. For callers that cannot
// allocate (graph capture, serving loops that forbid hipMalloc).
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace spmm {
namespace {

// Device scratch of the allocation-free entry point, one copy per GPU, held
// until the process ends. Layout (int32): [0] internal status, [1] entry count
// of the last call, then from word 64: row_ptr [mb + 1], col_idx [max_nnzb],
// csr_src [max_nnzb], panel_ptr [num_panels + 1].
constexpr int64_t kScratchInts = SPMM_NOALLOC_SCRATCH_BYTES / 4;
constexpr int64_t kScratchHead = 64;
static __device__ __align__(256) int32_t scratch[kScratchInts];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
int32_t* g_ptr[kMaxDevices] = {};  // device address of `scratch` on each device

// The device address of this device's scratch (hipGetSymbolAddress once per
// device, with that device current). Host code never uses the array's name as
// an address: only the pointer returned here reaches kernels.
spmm_status_t scratch_ptr(int device, int32_t** out) {
  if (device < 0 || device >= kMaxDevices) return fail(SPMM_ERR_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(SPMM_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_ptr[device] = (int32_t*)p;
  }
  *out = g_ptr[device];
  return SPMM_OK;
}

}  // namespace
}  // namespace spmm

using namespace spmm;

extern "C" spmm_status_t spmm_run_dynamic_noalloc(int64_t m, int64_t k, int32_t b, int64_t max_nnzb, spmm_dtype_t w,
                                                  spmm_dtype_t x, spmm_dtype_t y, const int32_t* nnzb_dev,
                                                  const int32_t* block_row_dev, const int32_t* block_col_dev,
                                                  const void* values_dev, const float* scales_dev, int64_t n,
                                                  const void* X, int64_t ldx, void* Y, int64_t ldy,
                                                  int32_t* status_dev, void* stream) {
  clear_error();
  if (m < 1 || k < 1) return fail(SPMM_ERR_INVALID_ARG, "m and k must be positive");
  if (b != 1 && b != 4 && b != 8 && b != 16 && b != 32)
    return fail(SPMM_ERR_INVALID_ARG, "block size must be one of 1, 4, 8, 16, 32");
  if (max_nnzb < 1) return fail(SPMM_ERR_INVALID_ARG, "max_nnzb must be positive");
  if (!dtype_triple_supported(w, x, y)) return fail(SPMM_ERR_UNSUPPORTED, "unsupported dtype combination");
  if (!nnzb_dev || !status_dev || !block_row_dev || !block_col_dev || !values_dev)
    return fail(SPMM_ERR_INVALID_ARG, "nnzb_dev, index, value and status buffers are required");
  if (w == SPMM_FP8_E4M3 && !scales_dev) return fail(SPMM_ERR_INVALID_ARG, "FP8 weights need block scales");
  if (w != SPMM_FP8_E4M3 && scales_dev) return fail(SPMM_ERR_INVALID_ARG, "block scales are only for FP8 weights");
  if (((uintptr_t)values_dev) % 16 != 0) return fail(SPMM_ERR_INVALID_ARG, "values are not 16-byte aligned");
  if (n < 0) return fail(SPMM_ERR_INVALID_ARG, "n is negative");
  if (n > INT32_MAX / 2 || m > INT32_MAX / 2 || k > INT32_MAX / 2)
    return fail(SPMM_ERR_UNSUPPORTED, "size too large");
  if (k % b != 0) return fail(SPMM_ERR_UNSUPPORTED, "the allocation-free path needs b to divide k");
  spmm_status_t st;
  if (n > 0) {
    if ((st = check_dense(X, ldx, n, dtype_bytes(x), "X")) != SPMM_OK) return st;
    if ((st = check_dense(Y, ldy, n, dtype_bytes(y), "Y")) != SPMM_OK) return st;
  }
  const int32_t mb = (int32_t)ceil_div(m, b), kb = (int32_t)ceil_div(k, b);
  // one row group per panel, as a dynamic handle made without options
  const Geometry geo = choose_geometry(m, k, b, max_nnzb, 0, nullptr, device_cu_count(), x);
  const int64_t need = kScratchHead + (int64_t)mb + 1 + 2 * max_nnzb + geo.num_panels + 1;
  if (need > kScratchInts)
    return fail(SPMM_ERR_CAPACITY, "the allocation-free path holds " + std::to_string(kScratchInts) +
                                       " int32 of scratch; this shape needs " + std::to_string(need));
  if (max_nnzb > INT32_MAX || !dynamic_small_fits((int32_t)max_nnzb, mb, kb, geo.num_groups))
    return fail(SPMM_ERR_CAPACITY, "capacity beyond the one-workgroup encoder of the allocation-free path");
  int device = 0;
  SPMM_HIP(hipGetDevice(&device));
  int32_t* base = nullptr;
  if ((st = scratch_ptr(device, &base)) != SPMM_OK) return st;
  int32_t* status = base;
  int32_t* nnz_last = base + 1;
  PlanBuffers pb;
  pb.row_ptr = base + kScratchHead;
  pb.col_idx = pb.row_ptr + mb + 1;
  pb.csr_src = pb.col_idx + max_nnzb;
  pb.panel_ptr = pb.csr_src + max_nnzb;
  hipStream_t s = (hipStream_t)stream;
  // the encoder writes every word the compute kernel reads (status included)
  st = build_dynamic_csr_small(nnzb_dev, block_row_dev, block_col_dev, (int32_t)max_nnzb, mb, kb, geo, pb, status,
                               status_dev, nnz_last, s);
  if (st != SPMM_OK || n == 0) return st;
  RunArgs a{};
  a.plan.m = (int32_t)m;
  a.plan.k = (int32_t)k;
  a.plan.b = b;
  a.plan.mb = mb;
  a.plan.kb = kb;
  a.plan.group_rows = geo.group_rows;
  a.plan.num_groups = geo.num_groups;
  a.plan.num_panels = geo.num_panels;
  a.plan.panel_ptr = pb.panel_ptr;
  a.plan.order = nullptr;
  a.W = values_dev;
  a.scales = scales_dev;
  a.w_index = pb.csr_src;
  a.X = X;
  a.Y = Y;
  a.ldx = ldx;
  a.ldy = ldy;
  a.n = (int32_t)n;
  a.wt = w;
  a.xt = x;
  a.yt = y;
  a.status = status;
  a.nnz = max_nnzb;
  return run_dynamic_kernel(a, pb.row_ptr, pb.col_idx, s);
}
