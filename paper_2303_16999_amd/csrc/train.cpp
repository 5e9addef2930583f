// Training-direction products (C ABI): the transposed plan, for the data
// gradient (M o W)^T dY, and the block-sampled product, for the weight
// gradient (dY X^T) o M.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <numeric>
#include <vector>

#include "internal.h"

using namespace spmm;

namespace {

// dst block e' = transpose of src block map[e'] (b x b, row-major); FP8 scales
// follow the same map.
template <typename T>
__global__ void k_transpose_blocks(const int32_t* __restrict__ map, int64_t nnz, int32_t b, const T* __restrict__ src,
                                   T* __restrict__ dst, const float* __restrict__ ssrc, float* __restrict__ sdst) {
  const int64_t bb = (int64_t)b * b;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nnz * bb; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i / bb, w = i - e * bb;
    const int32_t r = (int32_t)(w / b), c = (int32_t)(w % b);
    const int64_t s = map[e];
    dst[i] = src[s * bb + (int64_t)c * b + r];
    if (w == 0 && ssrc) sdst[e] = ssrc[s];
  }
}

// The tiled SDDMM reads a tile's dY and X rows once per task (2 kTile rows)
// where the per-block form reads each block's X rows and its row's dY rows
// (about 1.25 row slabs of 16 per b = 16 block, 3 per b = 32 block): it pays
// from about 24 blocks of 16 (8 of 32) per task. SPMM_SDDMM_TILED=0/1 forces
// the choice.
// The dense GEMM for the weight gradient where the mask is dense enough that
// a library GEMM of all of dY X^T and a gather beat the sampled products: the
// sampled kernels reach about 7.5, 30, 57, 193 and 240 TFLOP/s at b = 1, 4,
// 8, 16, 32 (m = k = 8192, n = 4096), the GEMM and gather about 1000 over the
// whole product, so the crossover densities are near their ratios
// (SPMM_SDDMM_DENSE=0/1 forces the choice).
bool sddmm_dense_preferred(const spmm_plan_s* p) {
  if (const char* e = getenv("SPMM_SDDMM_DENSE")) return e[0] == '1';
  if (p->mb < 1 || p->kb < 1) return false;
  const double d = (double)p->nnzb / ((double)p->mb * (double)p->kb);
  const double th = p->b == 1 ? 1.0 / 128 : p->b == 4 ? 1.0 / 32 : p->b == 8 ? 1.0 / 16 : p->b == 16 ? 3.0 / 16 : 0.25;
  return d >= th;
}

bool sddmm_tiled_preferred(const spmm_plan_s* p) {
  if (!p->sddmm_tiled_tasks || p->sddmm_tiled_num == 0) return false;
  if (const char* e = getenv("SPMM_SDDMM_TILED")) return e[0] == '1';
  return p->nnzb >= (int64_t)p->sddmm_tiled_num * (p->b == 16 ? 24 : 8);
}

}  // namespace

extern "C" {

spmm_status_t spmm_plan_transpose(spmm_plan_t p, const spmm_plan_opts* opts, spmm_plan_t* out) {
  clear_error();
  if (!out) return fail(SPMM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!p) return fail(SPMM_ERR_INVALID_ARG, "plan is NULL");
  if (!p->has_values) return fail(SPMM_ERR_INVALID_ARG, "values were not set on this plan");
  spmm_status_t st = check_device(p->device);
  if (st != SPMM_OK) return st;
  const int32_t mb = p->mb, kb = p->kb, b = p->b;
  const int64_t nnz = p->nnzb;
  std::vector<int32_t> rp((size_t)mb + 1), ci((size_t)std::max<int64_t>(nnz, 1));
  SPMM_HIP(hipMemcpy(rp.data(), p->pb.row_ptr, sizeof(int32_t) * rp.size(), hipMemcpyDeviceToHost));
  if (nnz) SPMM_HIP(hipMemcpy(ci.data(), p->pb.col_idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
  // block mask of W^T, and for each entry of its CSR (ordered by (c, r)) the source CSR entry
  std::vector<uint8_t> mask_t((size_t)kb * mb, 0);
  std::vector<int32_t> cnt((size_t)kb + 1, 0);
  for (int32_t r = 0; r < mb; ++r)
    for (int32_t q = rp[r]; q < rp[r + 1]; ++q) {
      mask_t[(size_t)ci[q] * mb + r] = 1;
      cnt[ci[q] + 1] += 1;
    }
  std::partial_sum(cnt.begin(), cnt.end(), cnt.begin());
  std::vector<int32_t> map((size_t)std::max<int64_t>(nnz, 1));
  for (int32_t r = 0; r < mb; ++r)  // rows ascending, so each column's entries come out by row
    for (int32_t q = rp[r]; q < rp[r + 1]; ++q) map[cnt[ci[q]]++] = q;
  spmm_plan_t t = nullptr;
  st = spmm_plan_static(p->k, p->m, b, mask_t.data(), p->w, p->x, p->y, opts, &t);
  if (st != SPMM_OK) return st;
  if (nnz == 0) {
    st = spmm_plan_set_values(t, nullptr, nullptr, nullptr);
    if (st != SPMM_OK) {
      spmm_plan_destroy(t);
      return st;
    }
    *out = t;
    return SPMM_OK;
  }
  const int eb = dtype_bytes(p->w);
  int32_t* map_dev = nullptr;
  void* vals = nullptr;
  float* scales = nullptr;
  hipError_t e = hipMalloc((void**)&map_dev, sizeof(int32_t) * nnz);
  if (e == hipSuccess) e = hipMalloc(&vals, (size_t)nnz * b * b * eb);
  if (e == hipSuccess && p->scales) e = hipMalloc((void**)&scales, sizeof(float) * nnz);
  if (e == hipSuccess) e = hipMemcpy(map_dev, map.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    const unsigned grid = (unsigned)std::min<int64_t>(8192, ceil_div(nnz * b * b, 256));
    if (eb == 1)
      hipLaunchKernelGGL(k_transpose_blocks<uint8_t>, dim3(grid), dim3(256), 0, nullptr, map_dev, nnz, b,
                         (const uint8_t*)p->values, (uint8_t*)vals, p->scales, scales);
    else if (eb == 2)
      hipLaunchKernelGGL(k_transpose_blocks<uint16_t>, dim3(grid), dim3(256), 0, nullptr, map_dev, nnz, b,
                         (const uint16_t*)p->values, (uint16_t*)vals, p->scales, scales);
    else
      hipLaunchKernelGGL(k_transpose_blocks<uint32_t>, dim3(grid), dim3(256), 0, nullptr, map_dev, nnz, b,
                         (const uint32_t*)p->values, (uint32_t*)vals, p->scales, scales);
    e = hipGetLastError();
  }
  if (e != hipSuccess) st = fail_hip(e, "transposed values");
  if (st == SPMM_OK) st = spmm_plan_set_values(t, vals, scales, nullptr);
  if (st == SPMM_OK && (e = hipDeviceSynchronize()) != hipSuccess) st = fail_hip(e, "transposed values");
  if (map_dev) (void)hipFree(map_dev);
  if (vals) (void)hipFree(vals);
  if (scales) (void)hipFree(scales);
  if (st != SPMM_OK) {
    spmm_plan_destroy(t);
    return st;
  }
  *out = t;
  return SPMM_OK;
}

spmm_status_t spmm_sddmm(spmm_plan_t p, int64_t n, const void* dY, int64_t lddy, const void* X, int64_t ldx,
                         float* G, void* stream) {
  clear_error();
  if (!p) return fail(SPMM_ERR_INVALID_ARG, "plan is NULL");
  if (n < 0) return fail(SPMM_ERR_INVALID_ARG, "n is negative");
  if (p->b > 32) return fail(SPMM_ERR_UNSUPPORTED, "SDDMM handles block sizes 1, 4, 8, 16 and 32");
  if (p->x != p->y || (p->x != SPMM_F16 && p->x != SPMM_BF16))
    return fail(SPMM_ERR_UNSUPPORTED, "SDDMM needs a plan with FP16 or BF16 X and Y");
  if (p->nnzb > 0 && !G) return fail(SPMM_ERR_INVALID_ARG, "G is NULL");
  if (n > INT32_MAX / 2) return fail(SPMM_ERR_UNSUPPORTED, "n too large");
  spmm_status_t st = check_device(p->device);
  if (st != SPMM_OK) return st;
  if (p->nnzb == 0) return SPMM_OK;
  if (n == 0) {  // an empty reduction: every block is zero
    SPMM_HIP(hipMemsetAsync(G, 0, sizeof(float) * (size_t)p->nnzb * p->b * p->b, (hipStream_t)stream));
    return SPMM_OK;
  }
  if ((st = check_dense(dY, lddy, n, 2, "dY")) != SPMM_OK) return st;
  if ((st = check_dense(X, ldx, n, 2, "X")) != SPMM_OK) return st;
  if (sddmm_dense_preferred(p) && n <= INT32_MAX && p->k <= INT32_MAX) {
    spmm_plan_s* q = const_cast<spmm_plan_s*>(p);
    const int64_t bytes = sddmm_dense_panel_rows(p) * p->k * 4;
    bool ws = q->sddmm_dense_ws_bytes >= bytes;
    if (!ws) {
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      if (hipStreamIsCapturing((hipStream_t)stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
        if (q->sddmm_dense_ws) {
          SPMM_HIP(hipDeviceSynchronize());
          (void)hipFree(q->sddmm_dense_ws);
          q->sddmm_dense_ws = nullptr;
          q->sddmm_dense_ws_bytes = 0;
        }
        if (hipMalloc((void**)&q->sddmm_dense_ws, (size_t)bytes) == hipSuccess) {
          q->sddmm_dense_ws_bytes = bytes;
          ws = true;
        } else {
          q->sddmm_dense_ws = nullptr;
        }
      }
    }
    if (ws) return sddmm_dense(p, n, dY, lddy, X, ldx, G, q->sddmm_dense_ws, (hipStream_t)stream);
  }
  if (sddmm_tiled_preferred(p))
    return launch_sddmm_tiled(p->x, p->b, p->sddmm_tiled_tasks, p->sddmm_tiled_ent, p->sddmm_tiled_num, p->m, p->k, n,
                              dY, lddy, X, ldx, G, (hipStream_t)stream);
  return launch_sddmm(p->x, p->b, p->pb.row_ptr, p->pb.col_idx, p->sddmm_tasks, p->sddmm_num_tasks, p->m, p->k, n, dY,
                      lddy, X, ldx, G, (hipStream_t)stream);
}

}  // extern "C"
