// Row-wise block-sparse x dense SpMM for FP32 W, X and Y (b = 16 or 32) on
// the 16x16x4 FP32 MFMA (PopSparse, Section 3: Y = (M o W) X; the paper's
// FP32 rows of Table 2).
//
// One wave owns one block row and 16*NS columns and walks the row's blocks in
// CSR order. For a block, MFMA t (t = 0 .. b/4 - 1) of row tile h takes k
// index g*(b/4) + t in lane group g: lane (g, i) then holds the b/4
// consecutive weights W[16h + i][g*b/4 ..] (one or two 16-byte loads), and
// lane (g, j) the X rows c*b + g*b/4 + t at columns n0 + NS*j .. + NS (one
// 8- or 16-byte load per row), so the lane's accumulators over s are NS
// consecutive columns of Y. No LDS and no barrier: the small FP32 problems
// this serves are latency-bound, and every block row and column tile gets its
// own wave.
#include "common.h"

namespace spmm {
namespace {

typedef float float2_t __attribute__((ext_vector_type(2)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr uint32_t kOOB = 0x80000000u;
constexpr int kRows = 4;  // block rows per workgroup, one per wave

struct P32 {
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const int32_t* w_index;  // dynamic mode: value block of each CSR entry (nullptr: the entry itself)
  const int32_t* status;   // dynamic mode: skip everything unless *status == 0 (nullptr: run)
  const float* W;
  const float* X;
  float* Y;
  int64_t ldx, ldy;
  int32_t m, k, n, mb;
  uint32_t x_bytes;
  int32_t relu;
  int32_t num_units;
};

__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int32_t xcd_unit(int32_t w, int32_t U) {
  const int32_t q = U >> 3, r = U & 7;
  const int32_t x = w & 7, local = w >> 3;
  return x * q + min(x, r) + local;
}

template <int NS>
__device__ __forceinline__ void load_x(__amdgpu_buffer_rsrc_t xr, int64_t row, int32_t k, int64_t ldx, int32_t col,
                                       float (&v)[NS]) {
  const uint32_t off = row < k ? (uint32_t)((row * ldx + col) * 4) : kOOB;
  if constexpr (NS == 4) {
    const float4_t t = __builtin_bit_cast(float4_t, __builtin_amdgcn_raw_buffer_load_b128(xr, off, 0, 0));
    v[0] = t[0]; v[1] = t[1]; v[2] = t[2]; v[3] = t[3];
  } else {
    const float2_t t = __builtin_bit_cast(float2_t, __builtin_amdgcn_raw_buffer_load_b64(xr, off, 0, 0));
    v[0] = t[0]; v[1] = t[1];
  }
}

template <int B, int NS>
__global__ __launch_bounds__(256) void k_spmm_row_f32(P32 p) {
  constexpr int H = B / 16, KS = B / 4;  // row tiles, MFMAs (k slices of one per lane group) per block
  if (p.status && *p.status) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  const int32_t unit = xcd_unit(blockIdx.x, p.num_units);
  const int32_t rgroups = (p.mb + kRows - 1) / kRows;
  const int32_t r = (unit % rgroups) * kRows + wave;
  if (r >= p.mb) return;
  const int32_t n0 = (unit / rgroups) * (16 * NS);
  const int32_t col = n0 + NS * j;
  __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)p.X, (short)0, (int)p.x_bytes, 0x00020000);
  float4_t acc[H][NS];
#pragma unroll
  for (int h = 0; h < H; ++h)
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[h][s] = float4_t{0.f, 0.f, 0.f, 0.f};
  const int32_t q_lo = uniform(p.row_ptr[r]), q_hi = uniform(p.row_ptr[r + 1]);
  for (int32_t q = q_lo; q < q_hi; ++q) {
    const int32_t c = uniform(p.col_idx[q]);
    const int64_t qv = p.w_index ? (int64_t)uniform(p.w_index[q]) : (int64_t)q;
    float xv[KS][NS];
#pragma unroll
    for (int t = 0; t < KS; ++t) load_x<NS>(xr, (int64_t)c * B + g * KS + t, p.k, p.ldx, col, xv[t]);
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const float* wrow = p.W + qv * B * B + (int64_t)(16 * h + j) * B + g * KS;
      float wv[KS];
#pragma unroll
      for (int t = 0; t < KS; t += 4) {
        const float4_t w4 = *(const float4_t*)(wrow + t);
        wv[t] = w4[0]; wv[t + 1] = w4[1]; wv[t + 2] = w4[2]; wv[t + 3] = w4[3];
      }
#pragma unroll
      for (int t = 0; t < KS; ++t)
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[h][s] = __builtin_amdgcn_mfma_f32_16x16x4f32(wv[t], xv[t][s], acc[h][s], 0, 0, 0);
    }
  }
  // lane (g, j) holds rows 4g + i (+16h) and columns col .. col + NS
#pragma unroll
  for (int h = 0; h < H; ++h)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = (int64_t)r * B + 16 * h + 4 * g + i;
      if (row >= p.m) continue;
      float v[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) v[s] = p.relu ? fmaxf(acc[h][s][i], 0.f) : acc[h][s][i];
      float* dst = p.Y + row * p.ldy + col;
      if (col + NS <= p.n) {
        if constexpr (NS == 4) *(float4_t*)dst = float4_t{v[0], v[1], v[2], v[3]};
        else *(float2_t*)dst = float2_t{v[0], v[1]};
      } else {
#pragma unroll
        for (int s = 0; s < NS; ++s)
          if (col + s < p.n) dst[s] = v[s];
      }
    }
}

}  // namespace

spmm_status_t launch_spmm_row_f32(const RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx, hipStream_t s) {
  if (a.plan.b != 16 && a.plan.b != 32) return fail(SPMM_ERR_UNSUPPORTED, "FP32 row-wise kernel handles b = 16 and 32");
  if ((int64_t)a.plan.k * a.ldx * 4 >= (int64_t)INT32_MAX)
    return fail(SPMM_ERR_UNSUPPORTED, "X larger than 2 GiB is not supported");
  const int ns = a.n > 32 ? 4 : 2;
  P32 p;
  p.row_ptr = row_ptr;
  p.col_idx = col_idx;
  p.w_index = a.w_index;
  p.status = a.status;
  p.W = (const float*)a.W;
  p.X = (const float*)a.X;
  p.Y = (float*)a.Y;
  p.ldx = a.ldx;
  p.ldy = a.ldy;
  p.m = a.plan.m;
  p.k = a.plan.k;
  p.n = a.n;
  p.mb = a.plan.mb;
  p.x_bytes = (uint32_t)((int64_t)a.plan.k * a.ldx * 4);
  p.relu = a.relu ? 1 : 0;
  const int64_t units = ceil_div(a.plan.mb, kRows) * ceil_div(a.n, 16 * ns);
  if (units == 0) return SPMM_OK;
  if (units > (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "too many work units");
  p.num_units = (int32_t)units;
  const dim3 grid((unsigned)units), block(256);
  if (a.plan.b == 16) {
    if (ns == 4) hipLaunchKernelGGL((k_spmm_row_f32<16, 4>), grid, block, 0, s, p);
    else hipLaunchKernelGGL((k_spmm_row_f32<16, 2>), grid, block, 0, s, p);
  } else {
    if (ns == 4) hipLaunchKernelGGL((k_spmm_row_f32<32, 4>), grid, block, 0, s, p);
    else hipLaunchKernelGGL((k_spmm_row_f32<32, 2>), grid, block, 0, s, p);
  }
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

}  // namespace spmm
