// Row-wise block-sparse x dense SpMM for grids with few workgroups per CU
// (PopSparse, Section 3: Y = (M o W) X), b = 16 and 32 with 16-bit W and X.
//
// The work split and the arithmetic are those of the row-wise kernel: one
// wave owns one block row and a tile of 16 NS columns, and pairs of
// consecutive blocks of the row fill one 16x16x32 MFMA, pair after pair in
// CSR order (for b = 32 each block is two such MFMAs per column tile), so the
// results are the same bit for bit. What differs is the
// schedule. With one or two waves per SIMD nothing hides the latency of a
// pair's loads, so the loop is software-pipelined over two pair buffers: the
// loads of the next pair are in flight while the current pair's MFMAs run.
// For the compiler to let them stay in flight, three things hold:
//   * the buffers keep the raw X rows and are transposed only at MFMA time
//     (a transpose right after the load would wait for it);
//   * every load is unconditional: past the end of the row the indices are
//     clamped and the X loads read out of range, which returns zeros, so the
//     number of loads in flight is the same on every path;
//   * the column (and value) indices of up to 64 blocks come from one vector
//     load per chunk and are broadcast with readlane, instead of a scalar load
//     per block whose wait would also wait for the loads in flight.
#include <cstdlib>

#include "spmm_row.h"

namespace spmm {
namespace {

using namespace row;

template <int NS>
struct PairBuf {
  u32x2 a1, a2;                             // A fragments of the pair's two blocks
  uint32_t x1[4][NS / 2], x2[4][NS / 2];    // raw X rows of the two blocks
};

template <int NS>
struct BlockBuf32 {
  u32x4 a[2];                               // A fragments of the block's two 16-row tiles
  uint32_t x1[4][NS / 2], x2[4][NS / 2];    // raw X rows 8g + i and 8g + 4 + i of the block
};

// Lane (g, j): X rows kr + 4g + i, columns n0 + NS j .. + NS, as loaded (no
// transpose); `valid` false reads zeros.
template <int NS>
__device__ __forceinline__ void xrows(__amdgpu_buffer_rsrc_t xr, const RowProblem& p, int32_t kr, bool valid, int g,
                                      int j, int32_t n0, uint32_t (&rows)[4][NS / 2]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t krow = (int64_t)kr + 4 * g + i;
    const uint32_t off = valid && krow < p.k ? (uint32_t)((krow * p.ldx + n0 + NS * j) * 2) : kOOB;
    if constexpr (NS == 8) {
      const u32x4 v = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(xr, off, 0, 0));
#pragma unroll
      for (int e = 0; e < 4; ++e) rows[i][e] = v[e];
    } else if constexpr (NS == 4) {
      const u32x2 v = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(xr, off, 0, 0));
      rows[i][0] = v.x;
      rows[i][1] = v.y;
    } else {
      rows[i][0] = __builtin_amdgcn_raw_buffer_load_b32(xr, off, 0, 0);
    }
  }
}

template <typename XT, int NS>
__device__ __forceinline__ void row_acc_pp(const RowProblem& p, int32_t q_lo, int32_t q_hi, int32_t n0, int lane,
                                           float4_t (&acc)[1][NS]) {
  constexpr int WB = 16 * 16 * 2;
  const int g = lane >> 4, j = lane & 15;
  __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)p.X, (short)0, (int)p.x_bytes, 0x00020000);
  const uint8_t* __restrict__ Wb = (const uint8_t*)p.W;
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[0][s] = float4_t{0.f, 0.f, 0.f, 0.f};
  for (int32_t c0 = q_lo; c0 < q_hi; c0 += 64) {
    const int32_t cn = min(64, q_hi - c0);
    const int32_t civ = lane < cn ? p.col_idx[c0 + lane] : 0;
    const int32_t wiv = p.w_index ? (lane < cn ? p.w_index[c0 + lane] : 0) : c0 + lane;
    // pair t (t even): blocks c0 + t and c0 + t + 1 of the chunk
    auto load = [&](int32_t t, PairBuf<NS>& B) {
      const int32_t t1 = min(t, cn - 1), t2 = min(t + 1, cn - 1);
      const int32_t c1 = __builtin_amdgcn_readlane(civ, t1), c2 = __builtin_amdgcn_readlane(civ, t2);
      const int64_t w1 = __builtin_amdgcn_readlane(wiv, t1), w2 = __builtin_amdgcn_readlane(wiv, t2);
      B.a1 = *(const u32x2*)(Wb + w1 * WB + (j * 16 + g * 4) * 2);
      B.a2 = *(const u32x2*)(Wb + w2 * WB + (j * 16 + g * 4) * 2);
      xrows<NS>(xr, p, c1 * 16, t < cn, g, j, n0, B.x1);
      xrows<NS>(xr, p, c2 * 16, t + 1 < cn, g, j, n0, B.x2);
    };
    auto mma = [&](int32_t t, const PairBuf<NS>& B) {
      u32x2 b1[NS], b2[NS];
      transpose4<NS>(B.x1, b1);
      transpose4<NS>(B.x2, b2);
      const bool two = t + 1 < cn;  // an odd last block: k slots 4-7 are zero
      const u32x4 a = u32x4{B.a1.x, B.a1.y, two ? B.a2.x : 0u, two ? B.a2.y : 0u};
#pragma unroll
      for (int s = 0; s < NS; ++s)
        acc[0][s] = Mma<XT>::k32(a, u32x4{b1[s].x, b1[s].y, b2[s].x, b2[s].y}, acc[0][s]);
    };
    PairBuf<NS> A, B;
    load(0, A);
    for (int32_t t = 0; t < cn; t += 4) {
      load(t + 2, B);
      mma(t, A);
      if (t + 2 >= cn) break;
      load(t + 4, A);
      mma(t + 2, B);
    }
  }
}

// b = 32: one block per MFMA step (two 16x16x32 MFMAs per column tile, one per
// 16-row tile), pipelined over two block buffers.
template <typename XT, int NS>
__device__ __forceinline__ void row_acc_pp32(const RowProblem& p, int32_t q_lo, int32_t q_hi, int32_t n0, int lane,
                                             float4_t (&acc)[2][NS]) {
  constexpr int WB = 32 * 32 * 2;
  const int g = lane >> 4, j = lane & 15;
  __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)p.X, (short)0, (int)p.x_bytes, 0x00020000);
  const uint8_t* __restrict__ Wb = (const uint8_t*)p.W;
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[h][s] = float4_t{0.f, 0.f, 0.f, 0.f};
  for (int32_t c0 = q_lo; c0 < q_hi; c0 += 64) {
    const int32_t cn = min(64, q_hi - c0);
    const int32_t civ = lane < cn ? p.col_idx[c0 + lane] : 0;
    const int32_t wiv = p.w_index ? (lane < cn ? p.w_index[c0 + lane] : 0) : c0 + lane;
    auto load = [&](int32_t t, BlockBuf32<NS>& B) {
      const int32_t tc = min(t, cn - 1);
      const int32_t c = __builtin_amdgcn_readlane(civ, tc);
      const int64_t w = __builtin_amdgcn_readlane(wiv, tc);
#pragma unroll
      for (int h = 0; h < 2; ++h) B.a[h] = *(const u32x4*)(Wb + w * WB + ((h * 16 + j) * 32 + g * 8) * 2);
      xrows<NS>(xr, p, c * 32, t < cn, 2 * g, j, n0, B.x1);
      xrows<NS>(xr, p, c * 32 + 4, t < cn, 2 * g, j, n0, B.x2);
    };
    auto mma = [&](const BlockBuf32<NS>& B) {
      u32x2 b1[NS], b2[NS];
      transpose4<NS>(B.x1, b1);
      transpose4<NS>(B.x2, b2);
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int s = 0; s < NS; ++s)
          acc[h][s] = Mma<XT>::k32(B.a[h], u32x4{b1[s].x, b1[s].y, b2[s].x, b2[s].y}, acc[h][s]);
    };
    BlockBuf32<NS> A, B;
    load(0, A);
    for (int32_t t = 0; t < cn; t += 2) {
      load(t + 1, B);
      mma(A);
      if (t + 1 >= cn) break;
      load(t + 2, A);
      mma(B);
    }
  }
}

template <typename XT, typename YT, int B, int NS>
__global__ __launch_bounds__(256) void k_spmm_row_pp(Params prm) {
  if (prm.status && *prm.status) return;
  const RowProblem& p = prm.pr;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int32_t unit = xcd_unit(blockIdx.x, prm.num_units);
  const int32_t rgroups = (p.mb + kRowsPerWg - 1) / kRowsPerWg;
  const int32_t r = (unit % rgroups) * kRowsPerWg + wave;
  if (r >= p.mb) return;
  const int32_t n0 = (unit / rgroups) * (16 * NS);
  const int32_t q_lo = uniform(p.row_ptr[r]), q_hi = uniform(p.row_ptr[r + 1]);
  float4_t acc[B / 16][NS];
  if constexpr (B == 16) row_acc_pp<XT, NS>(p, q_lo, q_hi, n0, lane, acc);
  else row_acc_pp32<XT, NS>(p, q_lo, q_hi, n0, lane, acc);
  row_store<YT, B, NS>(p, r, n0, lane, acc);
}

template <typename XT, typename YT, int B>
spmm_status_t launch_ns(const Params& prm, int ns, unsigned grid, hipStream_t s) {
  if (ns == 8) hipLaunchKernelGGL((k_spmm_row_pp<XT, YT, B, 8>), dim3(grid), dim3(256), 0, s, prm);
  else if (ns == 4) hipLaunchKernelGGL((k_spmm_row_pp<XT, YT, B, 4>), dim3(grid), dim3(256), 0, s, prm);
  else if (ns == 2) hipLaunchKernelGGL((k_spmm_row_pp<XT, YT, B, 2>), dim3(grid), dim3(256), 0, s, prm);
  else return fail(SPMM_ERR_INVALID_ARG, "column tile variant must be 2, 4 or 8");
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

template <int B>
spmm_status_t launch_xy(const RunArgs& a, const Params& prm, int ns, unsigned grid, hipStream_t s) {
  if (a.xt == SPMM_F16) {
    if (a.yt == SPMM_F32) return launch_ns<_Float16, float, B>(prm, ns, grid, s);
    return launch_ns<_Float16, _Float16, B>(prm, ns, grid, s);
  }
  if (a.yt == SPMM_F32) return launch_ns<__bf16, float, B>(prm, ns, grid, s);
  return launch_ns<__bf16, __bf16, B>(prm, ns, grid, s);
}

}  // namespace

// The pipelined schedule where it measured faster: launches of at most twice
// as many workgroups as CUs (at most two waves per SIMD; at four per SIMD
// the plain loop is as fast or faster) whose rows average at least 16 blocks
// of 16 (8 of 32): with 4 - 8 blocks of 16 a row is over before the pipeline
// fills, and the plain loop wins. SPMM_ROW_PP=0/1 forces the choice (for
// comparisons).
bool row_pp_preferred(int32_t b, int32_t mb, int64_t n, int32_t ns, int64_t nnz, int num_cus) {
  if (b != 16 && b != 32) return false;
  if (const char* e = getenv("SPMM_ROW_PP")) return e[0] == '1';
  return ceil_div(mb, kRowsPerWg) * ceil_div(n, 16 * ns) <= 2 * (int64_t)num_cus &&
         nnz >= (b == 16 ? 16 : 8) * (int64_t)mb;
}

bool split_all_preferred(int32_t b, int32_t mb, int64_t n, int32_t ns, int64_t nnz, int num_cus) {
  if (b != 16) return false;
  if (const char* e = getenv("SPMM_SPLIT_ALL")) return e[0] == '1';
  return ceil_div(mb, kRowsPerWg) * ceil_div(n, 16 * ns) <= 2 * (int64_t)num_cus && nnz >= 16 * (int64_t)mb;
}

spmm_status_t launch_spmm_row_pp(const RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx, hipStream_t s) {
  if (a.plan.b != 16 && a.plan.b != 32) return fail(SPMM_ERR_UNSUPPORTED, "pipelined row-wise kernel handles b = 16 and 32");
  if (a.wt == SPMM_FP8_E4M3 || a.wt != a.xt) return fail(SPMM_ERR_UNSUPPORTED, "pipelined row-wise kernel needs W in the X type");
  if ((int64_t)a.plan.k * a.ldx * 2 >= (int64_t)INT32_MAX)
    return fail(SPMM_ERR_UNSUPPORTED, "X larger than 2 GiB is not supported");
  Params prm;
  prm.pr = row::row_problem(a, row_ptr, col_idx);
  prm.pr.num_heavy = 0;
  prm.pr.light_rows = nullptr;
  prm.pr.num_light = a.plan.mb;
  prm.pr.heavy_rows = nullptr;
  prm.pr.part = nullptr;
  prm.status = a.status;
  const int ns = a.ns;
  if (ns != 2 && ns != 4 && ns != 8) return fail(SPMM_ERR_INVALID_ARG, "column tile variant must be 2, 4 or 8");
  const int64_t units = ceil_div(a.plan.mb, kRowsPerWg) * ceil_div(a.n, 16 * ns);
  if (units == 0) return SPMM_OK;
  if (units > (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "too many work units");
  prm.num_units = (int32_t)units;
  const unsigned grid = (unsigned)units;
  if (a.plan.b == 16) return launch_xy<16>(a, prm, ns, grid, s);
  return launch_xy<32>(a, prm, ns, grid, s);
}

}  // namespace spmm
