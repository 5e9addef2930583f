// Blocked-ELL input (C ABI): a pattern given as a fixed number of block-column
// slots per block row, -1 for an empty slot, becomes an ordinary plan; values
// given in slot order are gathered into the plan's block-CSR order on the
// device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "internal.h"

using namespace spmm;

namespace {

// dst block e = src slot slot[e] (b x b elements of T); FP8 scales likewise.
template <typename T>
__global__ void k_gather_slots(const int32_t* __restrict__ slot, int64_t nnz, int32_t bb, const T* __restrict__ src,
                               T* __restrict__ dst, const float* __restrict__ ssrc, float* __restrict__ sdst) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nnz * bb; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i / bb, w = i - e * bb;
    const int64_t s = slot[e];
    dst[i] = src[s * bb + w];
    if (w == 0 && ssrc) sdst[e] = ssrc[s];
  }
}

}  // namespace

extern "C" {

spmm_status_t spmm_plan_ell(int64_t m, int64_t k, int32_t b, int32_t ell_width, const int32_t* ell_cols_host,
                            spmm_dtype_t w, spmm_dtype_t x, spmm_dtype_t y, const spmm_plan_opts* opts,
                            spmm_plan_t* out) {
  clear_error();
  if (!out) return fail(SPMM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (m < 1 || k < 1 || b < 1) return fail(SPMM_ERR_INVALID_ARG, "m, k and b must be positive");
  if (ell_width < 0) return fail(SPMM_ERR_INVALID_ARG, "ELL width is negative");
  if (ell_width > 0 && !ell_cols_host) return fail(SPMM_ERR_INVALID_ARG, "ELL column array is NULL");
  const int64_t mb = ceil_div(m, b), kb = ceil_div(k, b);
  if (mb * kb > (int64_t)1 << 34) return fail(SPMM_ERR_UNSUPPORTED, "block grid too large");
  if (mb * (int64_t)ell_width > INT32_MAX / 2) return fail(SPMM_ERR_UNSUPPORTED, "ELL array too large");
  // the equivalent mask, and for each block (r, c) the slot that holds it
  std::vector<uint8_t> mask((size_t)(mb * kb), 0);
  std::vector<int32_t> where((size_t)(mb * kb), -1);
  for (int64_t r = 0; r < mb; ++r)
    for (int32_t s = 0; s < ell_width; ++s) {
      const int32_t c = ell_cols_host[r * ell_width + s];
      if (c == -1) continue;
      if (c < 0 || c >= kb) return fail(SPMM_ERR_INVALID_ARG, "ELL column index outside [-1, ceil(k/b))");
      if (mask[r * kb + c]) return fail(SPMM_ERR_INVALID_ARG, "a block column appears twice in one ELL row");
      mask[r * kb + c] = 1;
      where[r * kb + c] = (int32_t)(r * ell_width + s);
    }
  spmm_plan_t p = nullptr;
  spmm_status_t st = spmm_plan_static(m, k, b, mask.data(), w, x, y, opts, &p);
  if (st != SPMM_OK) return st;
  // slot of every CSR entry (rows ascending, columns ascending: the mask's row-major order)
  std::vector<int32_t> slot;
  slot.reserve((size_t)p->nnzb);
  for (int64_t i = 0; i < mb * kb; ++i)
    if (mask[i]) slot.push_back(where[i]);
  p->ell_width = ell_width;
  if (!slot.empty()) {
    hipError_t e = hipMalloc((void**)&p->ell_slot, sizeof(int32_t) * slot.size());
    if (e == hipSuccess) e = hipMemcpy(p->ell_slot, slot.data(), sizeof(int32_t) * slot.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      spmm_plan_destroy(p);
      return fail_hip(e, "ELL slot map");
    }
  }
  *out = p;
  return SPMM_OK;
}

spmm_status_t spmm_plan_set_values_ell(spmm_plan_t p, const void* values_ell_dev, const float* scales_ell_dev,
                                       void* stream) {
  clear_error();
  if (!p) return fail(SPMM_ERR_INVALID_ARG, "plan is NULL");
  if (p->ell_width == 0 && p->nnzb > 0) return fail(SPMM_ERR_INVALID_ARG, "plan was not built from blocked-ELL");
  if (p->nnzb > 0 && !values_ell_dev) return fail(SPMM_ERR_INVALID_ARG, "values are NULL");
  if (p->w == SPMM_FP8_E4M3 && p->nnzb > 0 && !scales_ell_dev)
    return fail(SPMM_ERR_INVALID_ARG, "FP8 weights need block scales");
  if (p->w != SPMM_FP8_E4M3 && scales_ell_dev) return fail(SPMM_ERR_INVALID_ARG, "block scales are only for FP8 weights");
  spmm_status_t st = check_device(p->device);
  if (st != SPMM_OK) return st;
  if (p->nnzb == 0) return spmm_plan_set_values(p, nullptr, nullptr, stream);
  hipStream_t s = (hipStream_t)stream;
  const int eb = dtype_bytes(p->w);
  const int32_t bb = p->b * p->b;
  void* tmp = nullptr;
  float* tmp_scales = nullptr;
  hipError_t e = hipMalloc(&tmp, (size_t)p->nnzb * bb * eb);
  if (e == hipSuccess && scales_ell_dev) e = hipMalloc((void**)&tmp_scales, sizeof(float) * p->nnzb);
  if (e == hipSuccess) {
    const unsigned grid = (unsigned)std::min<int64_t>(8192, ceil_div(p->nnzb * bb, 256));
    if (eb == 1)
      hipLaunchKernelGGL(k_gather_slots<uint8_t>, dim3(grid), dim3(256), 0, s, p->ell_slot, p->nnzb, bb,
                         (const uint8_t*)values_ell_dev, (uint8_t*)tmp, scales_ell_dev, tmp_scales);
    else if (eb == 2)
      hipLaunchKernelGGL(k_gather_slots<uint16_t>, dim3(grid), dim3(256), 0, s, p->ell_slot, p->nnzb, bb,
                         (const uint16_t*)values_ell_dev, (uint16_t*)tmp, scales_ell_dev, tmp_scales);
    else
      hipLaunchKernelGGL(k_gather_slots<uint32_t>, dim3(grid), dim3(256), 0, s, p->ell_slot, p->nnzb, bb,
                         (const uint32_t*)values_ell_dev, (uint32_t*)tmp, scales_ell_dev, tmp_scales);
    e = hipGetLastError();
  }
  if (e != hipSuccess) st = fail_hip(e, "ELL value gather");
  if (st == SPMM_OK) st = spmm_plan_set_values(p, tmp, tmp_scales, stream);
  // the temporaries are released once the work enqueued on `stream` is done
  e = hipStreamSynchronize(s);
  if (st == SPMM_OK && e != hipSuccess) st = fail_hip(e, "ELL value gather");
  if (tmp) (void)hipFree(tmp);
  if (tmp_scales) (void)hipFree(tmp_scales);
  return st;
}

}  // extern "C"
