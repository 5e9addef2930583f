// Dense dispatch. Section 5 of the paper summarises where a static sparse
// product beats a dense one by a power law in feature size, density and block
// size; this library refits that law to its own kernels (spmm_speedup_model).
// A plan created with dense dispatch asks the law at build time, and where it
// predicts the sparse kernels slower than a dense GEMM the plan keeps a dense
// copy of M o W (m x k, row-major, zeros outside the blocks) and its runs may
// use a library GEMM (rocBLAS, FP32 accumulation) on it. Whether they do is
// then measured by the autotuner like any other variant (form 3).
#include <rocblas/rocblas.h>

#include <map>
#include <mutex>

#include "internal.h"

namespace spmm {
namespace {

// Element i of the CSR values (entry e = i / b^2) to its place in the dense
// matrix; the block row of e is the last row whose first entry is <= e.
template <typename T>
__global__ void k_densify(const int32_t* __restrict__ row_ptr, int32_t mb, const int32_t* __restrict__ col_idx,
                          int64_t nnz, int32_t b, int64_t m, int64_t k, const T* __restrict__ vals,
                          T* __restrict__ dense) {
  const int64_t bb = (int64_t)b * b;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nnz * bb; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i / bb, w = i - e * bb;
    int32_t lo = 0, hi = mb - 1;
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (row_ptr[mid] <= e) lo = mid;
      else hi = mid - 1;
    }
    const int64_t row = (int64_t)lo * b + w / b, col = (int64_t)col_idx[e] * b + w % b;
    if (row < m && col < k) dense[row * k + col] = vals[i];
  }
}

rocblas_datatype rb_type(spmm_dtype_t t) {
  switch (t) {
    case SPMM_F16: return rocblas_datatype_f16_r;
    case SPMM_BF16: return rocblas_datatype_bf16_r;
    default: return rocblas_datatype_f32_r;
  }
}

std::mutex g_blas_mu;
std::map<int, rocblas_handle> g_blas;  // one handle per device, created on first use

}  // namespace

bool dense_dispatch_eligible(spmm_dtype_t w, spmm_dtype_t x, spmm_dtype_t y) {
  return w == x && (x == SPMM_F16 || x == SPMM_BF16) && (y == x || y == SPMM_F32);
}

spmm_status_t build_dense_copy(spmm_plan_s* p, hipStream_t s) {
  const size_t bytes = (size_t)p->m * (size_t)p->k * dtype_bytes(p->w);
  if (!p->dense_w) {
    hipError_t e = hipMalloc(&p->dense_w, bytes);
    if (e != hipSuccess) {
      p->dense_w = nullptr;
      return fail_hip(e, "hipMalloc dense copy");
    }
  }
  SPMM_HIP(hipMemsetAsync(p->dense_w, 0, bytes, s));
  if (p->nnzb == 0) return SPMM_OK;
  const unsigned grid = (unsigned)std::min<int64_t>(16384, ceil_div(p->nnzb * p->b * p->b, 256));
  hipLaunchKernelGGL(k_densify<uint16_t>, dim3(grid), dim3(256), 0, s, p->pb.row_ptr, p->mb, p->pb.col_idx, p->nnzb,
                     p->b, p->m, p->k, (const uint16_t*)p->values, (uint16_t*)p->dense_w);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

spmm_status_t run_dense(const spmm_plan_s* p, int64_t n, const void* X, int64_t ldx, void* Y, int64_t ldy,
                        hipStream_t s) {
  if (!p->dense_w) return fail(SPMM_ERR_INVALID_ARG, "the plan has no dense copy");
  std::lock_guard<std::mutex> lk(g_blas_mu);
  rocblas_handle& h = g_blas[p->device];
  if (!h && rocblas_create_handle(&h) != rocblas_status_success) {
    h = nullptr;
    return fail(SPMM_ERR_HIP, "rocblas_create_handle failed");
  }
  if (rocblas_set_stream(h, s) != rocblas_status_success) return fail(SPMM_ERR_HIP, "rocblas_set_stream failed");
  // column-major view: Y^T (n x m) = X^T (n x k) * Wd^T (k x m)
  const float alpha = 1.f, beta = 0.f;
  const rocblas_status r = rocblas_gemm_ex(h, rocblas_operation_none, rocblas_operation_none, (rocblas_int)n,
                                           (rocblas_int)p->m, (rocblas_int)p->k, &alpha, X, rb_type(p->x),
                                           (rocblas_int)ldx, p->dense_w, rb_type(p->w), (rocblas_int)p->k, &beta, Y,
                                           rb_type(p->y), (rocblas_int)ldy, Y, rb_type(p->y), (rocblas_int)ldy,
                                           rocblas_datatype_f32_r, rocblas_gemm_algo_standard, 0, 0);
  if (r != rocblas_status_success)
    return fail(SPMM_ERR_HIP, std::string("rocblas_gemm_ex failed: ") + rocblas_status_to_string(r));
  return SPMM_OK;
}

}  // namespace spmm

namespace spmm {
namespace {

// The blocks of block rows [r0, r0 + rb) of a plan, gathered from a dense FP32
// panel D (rows r0 * b .. of dY X^T, row-major, leading dimension k) into G in
// CSR order; zero outside m x k.
__global__ void k_gather_blocks(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx, int32_t r0,
                                int32_t rb, int32_t b, int64_t m, int64_t k, const float* __restrict__ D,
                                float* __restrict__ G) {
  const int32_t lo = row_ptr[r0], hi = row_ptr[r0 + rb];
  const int64_t bb = (int64_t)b * b;
  for (int64_t i = (int64_t)lo * bb + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)hi * bb;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i / bb, w = i - e * bb;
    int32_t a = r0, z = r0 + rb - 1;  // the block row of entry e: the last row whose first entry is <= e
    while (a < z) {
      const int32_t mid = (a + z + 1) >> 1;
      if (row_ptr[mid] <= e) a = mid;
      else z = mid - 1;
    }
    const int64_t row = (int64_t)a * b + w / b, col = (int64_t)col_idx[e] * b + w % b;
    G[i] = (row < m && col < k) ? D[(row - (int64_t)r0 * b) * k + col] : 0.f;
  }
}

}  // namespace

int64_t sddmm_dense_panel_rows(const spmm_plan_s* p) {
  const int64_t cap = (int64_t)128 << 20;  // bytes of one FP32 panel
  int64_t rows = std::max<int64_t>(p->b, cap / (4 * std::max<int64_t>(p->k, 1)));
  rows = std::min<int64_t>(rows, (int64_t)p->mb * p->b);
  return rows / p->b * p->b;
}

spmm_status_t sddmm_dense(const spmm_plan_s* p, int64_t n, const void* dY, int64_t lddy, const void* X, int64_t ldx,
                          float* G, float* ws, hipStream_t s) {
  const int64_t P = sddmm_dense_panel_rows(p);
  const int32_t pb = (int32_t)(P / p->b);
  std::lock_guard<std::mutex> lk(g_blas_mu);
  rocblas_handle& h = g_blas[p->device];
  if (!h && rocblas_create_handle(&h) != rocblas_status_success) {
    h = nullptr;
    return fail(SPMM_ERR_HIP, "rocblas_create_handle failed");
  }
  if (rocblas_set_stream(h, s) != rocblas_status_success) return fail(SPMM_ERR_HIP, "rocblas_set_stream failed");
  const float alpha = 1.f, beta = 0.f;
  const size_t eb = 2;  // FP16 / BF16 dY and X
  for (int32_t r0 = 0; r0 < p->mb; r0 += pb) {
    const int32_t rb = std::min<int32_t>(pb, p->mb - r0);
    const int64_t rows = std::min<int64_t>((int64_t)rb * p->b, p->m - (int64_t)r0 * p->b);
    // column-major view: the panel's (dY X^T)^T (k x rows) = X (k x n, X^T stored) * dY^T (n x rows)
    const void* dYp = (const uint8_t*)dY + (size_t)r0 * p->b * lddy * eb;
    const rocblas_status r =
        rocblas_gemm_ex(h, rocblas_operation_transpose, rocblas_operation_none, (rocblas_int)p->k, (rocblas_int)rows,
                        (rocblas_int)n, &alpha, X, rb_type(p->x), (rocblas_int)ldx, dYp, rb_type(p->x),
                        (rocblas_int)lddy, &beta, ws, rocblas_datatype_f32_r, (rocblas_int)p->k, ws,
                        rocblas_datatype_f32_r, (rocblas_int)p->k, rocblas_datatype_f32_r, rocblas_gemm_algo_standard, 0,
                        0);
    if (r != rocblas_status_success)
      return fail(SPMM_ERR_HIP, std::string("rocblas_gemm_ex failed: ") + rocblas_status_to_string(r));
    const unsigned grid = (unsigned)std::min<int64_t>(65536, ceil_div(p->nnzb * p->b * p->b, 256));
    hipLaunchKernelGGL(k_gather_blocks, dim3(grid), dim3(256), 0, s, p->pb.row_ptr, p->pb.col_idx, r0, rb, p->b, p->m,
                       p->k, (const float*)ws, G);
    SPMM_HIP(hipGetLastError());
  }
  return SPMM_OK;
}

}  // namespace spmm
