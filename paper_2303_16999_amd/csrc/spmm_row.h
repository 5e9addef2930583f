// Row-wise block-sparse x dense SpMM for 16-bit X (FP16/BF16), block sizes 16
// and 32, weights in FP16/BF16 or FP8-E4M3 with per-block FP32 scales.
//
// Y = (M o W) * X (PopSparse, Section 3), FP32 accumulation.
//
// One wave owns one block row and a tile of 16*NS columns and walks the row's
// nonzero blocks in block-CSR order. There is no LDS and no barrier: every
// wave is independent, and the latency of its loads is hidden by the other
// waves resident on the SIMD (the kernel keeps its registers small enough for
// four waves per SIMD). For each block the wave loads
//   * its A fragment, W[row][k-range] (8 or 16 bytes per lane, one contiguous
//     512-byte read per wave for a b = 16 block), and
//   * its B fragments: lane (g, j) reads 16 bytes of X along n from each of the
//     k rows its lane group covers and transposes them in registers (v_perm),
//     so column j of MFMA tile s is physical column 8*j + s of the tile and
//     the lane ends up holding 8 consecutive output columns per row.
// Consecutive b = 16 blocks of the row are fused into one 16x16x32 MFMA.
// Buffer loads return zero out of range, which covers the k and n tails.
// Workgroups are ordered so that the rows of one n-tile run on one XCD at the
// same time: the X columns they share stay in that XCD's L2.
#pragma once

#include "common.h"

namespace spmm {
namespace row {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef float float2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct Fp8 {};  // weights stored as OCP E4M3FN codes

// One SpMM as the row-wise kernel sees it (also an entry of the grouped
// launch's descriptor table in device memory).
struct RowProblem {
  const int32_t* row_ptr;  // [mb + 1]
  const int32_t* col_idx;  // [nnz]
  const void* W;           // values in block-CSR order (or indexed by w_index)
  const float* scales;     // FP8 block scales, indexed like W, else nullptr
  const int32_t* w_index;  // entry q's values are block w_index[q] of W; nullptr: block q
  const void* X;
  void* Y;
  int64_t ldx, ldy;
  int32_t m, k, n, mb;
  uint32_t x_bytes;        // k * ldx * 2, < 2^31
  int32_t relu;            // nonzero: max(0, y) before the output cast
  int32_t ns;              // column tiles of 16 per wave: 2, 4 or 8
  int32_t unit_begin;      // grouped launch: first workgroup of this problem (a multiple of 8)
  int32_t num_heavy;       // split rows (or pieces, with part set): heavy units per column tile
  int32_t num_units;       // grouped launch: work units of this problem
  const int32_t* light_rows;  // [num_light] the rows light units take, in that order; nullptr: all rows in order
  // part == nullptr: [num_heavy] the split rows (nullptr with num_heavy == mb:
  // every row, in order). part set: [num_heavy][8] pieces (piece_store).
  const int32_t* heavy_rows;
  float* part;             // piece partial sums, nullptr: no pieces
  int32_t num_light;       // rows of the light units
  int32_t row_slices;      // nonzero: light units ordered by eighths of their row groups (light_unit)
};

struct Params {
  RowProblem pr;
  int32_t num_units;
  const int32_t* status;   // skip when *status != 0 (dynamic), else nullptr
};

constexpr int kRowsPerWg = 4;  // one block row per wave

constexpr uint32_t kOOB = 0x80000000u;

__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Wave-uniform load of an index array that no kernel writes while it runs,
// through the constant address space: it stays a scalar load (which does not
// wait for the vector loads in flight) in kernels with a barrier, where the
// compiler cannot prove the memory unchanged.
__device__ __forceinline__ int32_t sload(const int32_t* base, int64_t i) {
  typedef const __attribute__((address_space(4))) int32_t* cptr;
  return uniform(((cptr)base)[i]);
}

__device__ __forceinline__ int32_t xcd_unit(int32_t w, int32_t U) {
  const int32_t q = U >> 3, r = U & 7;
  const int32_t x = w & 7, local = w >> 3;
  return x * q + min(x, r) + local;
}

template <typename XT> struct Mma;
template <> struct Mma<_Float16> {
  static __device__ __forceinline__ float4_t k32(u32x4 a, u32x4 b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(half8_t, a), __builtin_bit_cast(half8_t, b), c, 0, 0, 0);
  }
  static __device__ __forceinline__ float4_t k16(u32x2 a, u32x2 b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(half4_t, a), __builtin_bit_cast(half4_t, b), c, 0, 0, 0);
  }
  static __device__ __forceinline__ uint32_t pack2(float lo, float hi) {
    _Float16 a = (_Float16)lo, b = (_Float16)hi;
    return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
  }
};
template <> struct Mma<__bf16> {
  static __device__ __forceinline__ float4_t k32(u32x4 a, u32x4 b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
  }
  static __device__ __forceinline__ float4_t k16(u32x2 a, u32x2 b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(short4_t, a), __builtin_bit_cast(short4_t, b), c, 0, 0, 0);
  }
  static __device__ __forceinline__ uint32_t pack2(float lo, float hi) {
    __bf16 a = (__bf16)lo, b = (__bf16)hi;
    return (uint32_t)__builtin_bit_cast(uint16_t, a) | ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
  }
};

template <typename XT>
__device__ __forceinline__ u32x2 fp8x4(uint32_t codes) {
  auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)codes, false);
  auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)codes, true);
  return u32x2{Mma<XT>::pack2(lo[0], lo[1]), Mma<XT>::pack2(hi[0], hi[1])};
}

template <typename YT> __device__ __forceinline__ YT to_out(float v);
template <> __device__ __forceinline__ float to_out<float>(float v) { return v; }
template <> __device__ __forceinline__ _Float16 to_out<_Float16>(float v) { return (_Float16)v; }
template <> __device__ __forceinline__ __bf16 to_out<__bf16>(float v) { return (__bf16)v; }

// Four X rows x NS columns (NS/2 dwords each) -> for each of the NS columns,
// the four k values as two dwords (k0,k1) (k2,k3). r[i] holds row i.
template <int NS>
__device__ __forceinline__ void transpose4(const uint32_t (&r)[4][NS / 2], u32x2 (&out)[NS]) {
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    const uint32_t sel = (q & 1) ? 0x07060302u : 0x05040100u;
    out[q].x = __builtin_amdgcn_perm(r[1][q >> 1], r[0][q >> 1], sel);
    out[q].y = __builtin_amdgcn_perm(r[3][q >> 1], r[2][q >> 1], sel);
  }
}

// lane (g, j): X rows kr + 4g + i (i = 0..3) for columns n0 + NS*j .. +NS, transposed
template <int NS>
__device__ __forceinline__ void xfrag(__amdgpu_buffer_rsrc_t xr, const RowProblem& p, int32_t kr, int g, int j,
                                      int32_t n0, u32x2 (&out)[NS]) {
  uint32_t rows[4][NS / 2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t krow = (int64_t)kr + 4 * g + i;
    const uint32_t off = krow < p.k ? (uint32_t)((krow * p.ldx + n0 + NS * j) * 2) : kOOB;
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
  transpose4<NS>(rows, out);
}

// Where a wave finds entry q of the row it walks: its block column and the
// block of W that holds its values. CsrIndex reads the plan's arrays (col_idx,
// and w_index when the values are not in CSR order); LdsKeys reads a sorted
// list of (column << 16 | input index) keys in LDS (the one-launch dynamic
// call, whose values stay in input order).
struct CsrIndex {
  const int32_t* col;
  const int32_t* widx;
  __device__ __forceinline__ int32_t column(int32_t q) const { return sload(col, q); }
  __device__ __forceinline__ int64_t block(int32_t q) const { return widx ? (int64_t)sload(widx, q) : (int64_t)q; }
};
struct LdsKeys {
  const uint32_t* keys;
  __device__ __forceinline__ int32_t column(int32_t q) const { return uniform((int32_t)(keys[q] >> 16)); }
  __device__ __forceinline__ int64_t block(int32_t q) const { return (int64_t)uniform((int32_t)(keys[q] & 0xffffu)); }
};

// Accumulates the blocks q_lo .. q_hi of one block row (in CSR order) for
// columns n0 .. n0 + 16*NS into acc (one wave; acc starts at zero).
template <typename XT, typename WT, int B, int NS, typename IX = CsrIndex, int PFX = 8 / NS>
__device__ __forceinline__ void row_acc(const RowProblem& p, int32_t q_lo, int32_t q_hi, int32_t n0, int lane,
                                        float4_t (&acc)[B / 16][NS], IX ix = IX{nullptr, nullptr}) {
  static_assert(NS == 2 || NS == 4 || NS == 8, "column tiles per wave");
  constexpr bool kFp8 = __is_same(WT, Fp8);
  constexpr int WB = B * B * (kFp8 ? 1 : 2);  // bytes per block
  constexpr int H = B / 16;
  const int g = lane >> 4, j = lane & 15;
  __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)p.X, (short)0, (int)p.x_bytes, 0x00020000);
  const uint8_t* __restrict__ Wb = (const uint8_t*)p.W;
#pragma unroll
  for (int h = 0; h < H; ++h)
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[h][s] = float4_t{0.f, 0.f, 0.f, 0.f};
  if constexpr (__is_same(IX, CsrIndex)) ix = CsrIndex{p.col_idx, p.w_index};
  auto wq = [&](int32_t q) -> int64_t { return ix.block(q); };
  if constexpr (!kFp8 && B == 16) {
    // pairs of blocks: k slots 0-3 from the first block, 4-7 from the second.
    // PF pairs are loaded before their MFMAs (more loads in flight where the
    // column tile, and so each pair's register footprint, is narrow); the
    // MFMAs still run pair after pair, so the sums do not depend on PF.
    constexpr int PF = PFX;
    for (int32_t q0 = q_lo; q0 < q_hi; q0 += 2 * PF) {
      u32x4 a[PF];
      u32x2 b1[PF][NS], b2[PF][NS];
#pragma unroll
      for (int f = 0; f < PF; ++f) {
        const int32_t q = q0 + 2 * f;
        if (f > 0 && q >= q_hi) break;
        const bool two = q + 1 < q_hi;
        const int32_t c1 = ix.column(q);
        const int32_t c2 = two ? ix.column(q + 1) : c1;
        const u32x2 a1 = *(const u32x2*)(Wb + wq(q) * WB + (j * 16 + g * 4) * 2);
        const u32x2 a2 = two ? *(const u32x2*)(Wb + wq(q + 1) * WB + (j * 16 + g * 4) * 2) : u32x2{0u, 0u};
        a[f] = u32x4{a1.x, a1.y, a2.x, a2.y};
        xfrag<NS>(xr, p, c1 * 16, g, j, n0, b1[f]);
        if (two) {
          xfrag<NS>(xr, p, c2 * 16, g, j, n0, b2[f]);
        } else {
#pragma unroll
          for (int s = 0; s < NS; ++s) b2[f][s] = u32x2{0u, 0u};
        }
      }
#pragma unroll
      for (int f = 0; f < PF; ++f) {
        if (f > 0 && q0 + 2 * f >= q_hi) break;
#pragma unroll
        for (int s = 0; s < NS; ++s)
          acc[0][s] = Mma<XT>::k32(a[f], u32x4{b1[f][s].x, b1[f][s].y, b2[f][s].x, b2[f][s].y}, acc[0][s]);
      }
    }
  } else if constexpr (!kFp8) {  // B == 32: k slots 0-3 and 4-7 are rows 8g..8g+3 and 8g+4..8g+7
    for (int32_t q = q_lo; q < q_hi; ++q) {
      const int32_t c = ix.column(q);
      u32x2 b1[NS], b2[NS];
      xfrag<NS>(xr, p, c * 32, 2 * g, j, n0, b1);      // rows c*32 + 8g + i
      xfrag<NS>(xr, p, c * 32 + 4, 2 * g, j, n0, b2);  // rows c*32 + 8g + 4 + i
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const u32x4 a = *(const u32x4*)(Wb + wq(q) * WB + ((h * 16 + j) * 32 + g * 8) * 2);
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[h][s] = Mma<XT>::k32(a, u32x4{b1[s].x, b1[s].y, b2[s].x, b2[s].y}, acc[h][s]);
      }
    }
  } else {  // FP8 weights with a per-block scale
    for (int32_t q = q_lo; q < q_hi; ++q) {
      const int32_t c = ix.column(q);
      const int64_t qv = wq(q);
      const float sc = p.scales[qv];
      if constexpr (B == 16) {
        const u32x2 a = fp8x4<XT>(*(const uint32_t*)(Wb + qv * WB + j * 16 + g * 4));
        u32x2 bx[NS];
        xfrag<NS>(xr, p, c * 16, g, j, n0, bx);
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[0][s] += sc * Mma<XT>::k16(a, bx[s], float4_t{0.f, 0.f, 0.f, 0.f});
      } else {
        u32x2 b1[NS], b2[NS];
        xfrag<NS>(xr, p, c * 32, 2 * g, j, n0, b1);
        xfrag<NS>(xr, p, c * 32 + 4, 2 * g, j, n0, b2);
#pragma unroll
        for (int h = 0; h < H; ++h) {
          const u32x2 codes = *(const u32x2*)(Wb + qv * WB + (h * 16 + j) * 32 + g * 8);
          const u32x2 lo = fp8x4<XT>(codes.x), hi = fp8x4<XT>(codes.y);
          const u32x4 a = {lo.x, lo.y, hi.x, hi.y};
#pragma unroll
          for (int s = 0; s < NS; ++s)
            acc[h][s] += sc * Mma<XT>::k32(a, u32x4{b1[s].x, b1[s].y, b2[s].x, b2[s].y}, float4_t{0.f, 0.f, 0.f, 0.f});
        }
      }
    }
  }

}

// Stores one wave's accumulators for block row r: lane (g, j) holds rows
// 4g + i (+16h) and columns n0 + NS*j .. +NS.
template <typename YT, int B, int NS>
__device__ __forceinline__ void row_store(const RowProblem& p, int32_t r, int32_t n0, int lane,
                                          float4_t (&acc)[B / 16][NS]) {
  constexpr int H = B / 16;
  const int g = lane >> 4, j = lane & 15;
  if (p.relu) {
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[h][s][i] = acc[h][s][i] > 0.f ? acc[h][s][i] : 0.f;
  }
  YT* __restrict__ Y = (YT*)p.Y;
  const int32_t col0 = n0 + NS * j;
#pragma unroll
  for (int h = 0; h < H; ++h) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = (int64_t)r * B + h * 16 + 4 * g + i;
      if (row >= p.m) continue;
      YT* dst = Y + row * p.ldy + col0;
      if (col0 + NS <= p.n) {
        if constexpr (sizeof(YT) == 4 && NS == 2) {
          const float v0 = acc[h][0][i], v1 = acc[h][1][i];
          *(float2_t*)dst = float2_t{v0, v1};
        } else if constexpr (sizeof(YT) == 4) {
#pragma unroll
          for (int s = 0; s < NS; s += 4) {
            const float v0 = acc[h][s][i], v1 = acc[h][s + 1][i], v2 = acc[h][s + 2][i], v3 = acc[h][s + 3][i];
            *(float4_t*)(dst + s) = float4_t{v0, v1, v2, v3};
          }
        } else {
          uint32_t w[NS / 2];
#pragma unroll
          for (int e = 0; e < NS / 2; ++e) {
            const float lo = acc[h][2 * e][i], hi = acc[h][2 * e + 1][i];
            w[e] = Mma<YT>::pack2(lo, hi);
          }
          if constexpr (NS == 8) *(u32x4*)dst = u32x4{w[0], w[1], w[2], w[3]};
          else if constexpr (NS == 4) *(u32x2*)dst = u32x2{w[0], w[1]};
          else *(uint32_t*)dst = w[0];
        }
      } else {
#pragma unroll
        for (int s = 0; s < NS; ++s)
          if (col0 + s < p.n) {
            const float v = acc[h][s][i];
            dst[s] = to_out<YT>(v);
          }
      }
    }
  }
}

// The work of one wave in a launch without split rows: block row r of
// problem p, columns n0 .. n0 + 16*NS. (The same steps as row_acc followed by
// row_store, kept in one body: split into the two, the compiler schedules the
// main loop differently and the kernel measured 3-6% slower.)
template <typename XT, typename WT, typename YT, int B, int NS>
__device__ __forceinline__ void row_tile_whole(const RowProblem& p, int32_t r, int32_t n0, int lane) {
  static_assert(NS == 2 || NS == 4 || NS == 8, "column tiles per wave");
  constexpr bool kFp8 = __is_same(WT, Fp8);
  constexpr int WB = B * B * (kFp8 ? 1 : 2);  // bytes per block
  constexpr int H = B / 16;
  const int g = lane >> 4, j = lane & 15;
  __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)p.X, (short)0, (int)p.x_bytes, 0x00020000);
  const uint8_t* __restrict__ Wb = (const uint8_t*)p.W;
  float4_t acc[H][NS];
#pragma unroll
  for (int h = 0; h < H; ++h)
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[h][s] = float4_t{0.f, 0.f, 0.f, 0.f};

  const int32_t q_lo = uniform(p.row_ptr[r]), q_hi = uniform(p.row_ptr[r + 1]);
  const int32_t* __restrict__ widx = p.w_index;
  auto wq = [&](int32_t q) -> int64_t { return widx ? (int64_t)uniform(widx[q]) : (int64_t)q; };
  if constexpr (!kFp8 && B == 16) {
    // pairs of blocks: k slots 0-3 from the first block, 4-7 from the second.
    // PF pairs are loaded before their MFMAs (more loads in flight where the
    // column tile, and so each pair's register footprint, is narrow); the
    // MFMAs still run pair after pair, so the sums do not depend on PF.
    constexpr int PF = 8 / NS;
    for (int32_t q0 = q_lo; q0 < q_hi; q0 += 2 * PF) {
      u32x4 a[PF];
      u32x2 b1[PF][NS], b2[PF][NS];
#pragma unroll
      for (int f = 0; f < PF; ++f) {
        const int32_t q = q0 + 2 * f;
        if (f > 0 && q >= q_hi) break;
        const bool two = q + 1 < q_hi;
        const int32_t c1 = uniform(p.col_idx[q]);
        const int32_t c2 = two ? uniform(p.col_idx[q + 1]) : c1;
        const u32x2 a1 = *(const u32x2*)(Wb + wq(q) * WB + (j * 16 + g * 4) * 2);
        const u32x2 a2 = two ? *(const u32x2*)(Wb + wq(q + 1) * WB + (j * 16 + g * 4) * 2) : u32x2{0u, 0u};
        a[f] = u32x4{a1.x, a1.y, a2.x, a2.y};
        xfrag<NS>(xr, p, c1 * 16, g, j, n0, b1[f]);
        if (two) {
          xfrag<NS>(xr, p, c2 * 16, g, j, n0, b2[f]);
        } else {
#pragma unroll
          for (int s = 0; s < NS; ++s) b2[f][s] = u32x2{0u, 0u};
        }
      }
#pragma unroll
      for (int f = 0; f < PF; ++f) {
        if (f > 0 && q0 + 2 * f >= q_hi) break;
#pragma unroll
        for (int s = 0; s < NS; ++s)
          acc[0][s] = Mma<XT>::k32(a[f], u32x4{b1[f][s].x, b1[f][s].y, b2[f][s].x, b2[f][s].y}, acc[0][s]);
      }
    }
  } else if constexpr (!kFp8) {  // B == 32: k slots 0-3 and 4-7 are rows 8g..8g+3 and 8g+4..8g+7
    for (int32_t q = q_lo; q < q_hi; ++q) {
      const int32_t c = uniform(p.col_idx[q]);
      u32x2 b1[NS], b2[NS];
      xfrag<NS>(xr, p, c * 32, 2 * g, j, n0, b1);      // rows c*32 + 8g + i
      xfrag<NS>(xr, p, c * 32 + 4, 2 * g, j, n0, b2);  // rows c*32 + 8g + 4 + i
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const u32x4 a = *(const u32x4*)(Wb + wq(q) * WB + ((h * 16 + j) * 32 + g * 8) * 2);
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[h][s] = Mma<XT>::k32(a, u32x4{b1[s].x, b1[s].y, b2[s].x, b2[s].y}, acc[h][s]);
      }
    }
  } else {  // FP8 weights with a per-block scale
    for (int32_t q = q_lo; q < q_hi; ++q) {
      const int32_t c = uniform(p.col_idx[q]);
      const int64_t qv = wq(q);
      const float sc = p.scales[qv];
      if constexpr (B == 16) {
        const u32x2 a = fp8x4<XT>(*(const uint32_t*)(Wb + qv * WB + j * 16 + g * 4));
        u32x2 bx[NS];
        xfrag<NS>(xr, p, c * 16, g, j, n0, bx);
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[0][s] += sc * Mma<XT>::k16(a, bx[s], float4_t{0.f, 0.f, 0.f, 0.f});
      } else {
        u32x2 b1[NS], b2[NS];
        xfrag<NS>(xr, p, c * 32, 2 * g, j, n0, b1);
        xfrag<NS>(xr, p, c * 32 + 4, 2 * g, j, n0, b2);
#pragma unroll
        for (int h = 0; h < H; ++h) {
          const u32x2 codes = *(const u32x2*)(Wb + qv * WB + (h * 16 + j) * 32 + g * 8);
          const u32x2 lo = fp8x4<XT>(codes.x), hi = fp8x4<XT>(codes.y);
          const u32x4 a = {lo.x, lo.y, hi.x, hi.y};
#pragma unroll
          for (int s = 0; s < NS; ++s)
            acc[h][s] += sc * Mma<XT>::k32(a, u32x4{b1[s].x, b1[s].y, b2[s].x, b2[s].y}, float4_t{0.f, 0.f, 0.f, 0.f});
        }
      }
    }
  }

  // epilogue: lane (g, j) holds rows 4g + i and columns n0 + NS*j .. +NS
  if (p.relu) {
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[h][s][i] = acc[h][s][i] > 0.f ? acc[h][s][i] : 0.f;
  }
  YT* __restrict__ Y = (YT*)p.Y;
  const int32_t col0 = n0 + NS * j;
#pragma unroll
  for (int h = 0; h < H; ++h) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = (int64_t)r * B + h * 16 + 4 * g + i;
      if (row >= p.m) continue;
      YT* dst = Y + row * p.ldy + col0;
      if (col0 + NS <= p.n) {
        if constexpr (sizeof(YT) == 4 && NS == 2) {
          const float v0 = acc[h][0][i], v1 = acc[h][1][i];
          *(float2_t*)dst = float2_t{v0, v1};
        } else if constexpr (sizeof(YT) == 4) {
#pragma unroll
          for (int s = 0; s < NS; s += 4) {
            const float v0 = acc[h][s][i], v1 = acc[h][s + 1][i], v2 = acc[h][s + 2][i], v3 = acc[h][s + 3][i];
            *(float4_t*)(dst + s) = float4_t{v0, v1, v2, v3};
          }
        } else {
          uint32_t w[NS / 2];
#pragma unroll
          for (int e = 0; e < NS / 2; ++e) {
            const float lo = acc[h][2 * e][i], hi = acc[h][2 * e + 1][i];
            w[e] = Mma<YT>::pack2(lo, hi);
          }
          if constexpr (NS == 8) *(u32x4*)dst = u32x4{w[0], w[1], w[2], w[3]};
          else if constexpr (NS == 4) *(u32x2*)dst = u32x2{w[0], w[1]};
          else *(uint32_t*)dst = w[0];
        }
      } else {
#pragma unroll
        for (int s = 0; s < NS; ++s)
          if (col0 + s < p.n) {
            const float v = acc[h][s][i];
            dst[s] = to_out<YT>(v);
          }
      }
    }
  }
}

// b = 64: the four waves of a workgroup share block row r, wave h computing
// its rows 16h .. 16h + 15 for columns n0 .. n0 + 16*NS. A block is two K = 32
// slices (k rows 32t .. 32t + 31; in a slice, k slots 0-3 and 4-7 are rows
// 8g .. 8g + 3 and 8g + 4 .. 8g + 7). The four waves read the same X slabs at
// about the same time, so the CU's L1 serves most of the repeats. FP8 blocks
// keep an FP32 partial over both slices and scale it.
template <typename XT, typename WT, typename YT, int NS>
__device__ __forceinline__ void row_tile_b64(const RowProblem& p, int32_t r, int h, int32_t n0, int lane) {
  constexpr bool kFp8 = __is_same(WT, Fp8);
  constexpr int WB = 64 * 64 * (kFp8 ? 1 : 2);  // bytes per block
  const int g = lane >> 4, j = lane & 15;
  __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)p.X, (short)0, (int)p.x_bytes, 0x00020000);
  const uint8_t* __restrict__ Wb = (const uint8_t*)p.W;
  float4_t acc[1][NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[0][s] = float4_t{0.f, 0.f, 0.f, 0.f};
  const int32_t q_lo = uniform(p.row_ptr[r]), q_hi = uniform(p.row_ptr[r + 1]);
  const int32_t* __restrict__ widx = p.w_index;
  for (int32_t q = q_lo; q < q_hi; ++q) {
    const int32_t c = uniform(p.col_idx[q]);
    const int64_t qv = widx ? (int64_t)uniform(widx[q]) : (int64_t)q;
    u32x2 b1[2][NS], b2[2][NS];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      xfrag<NS>(xr, p, c * 64 + 32 * t, 2 * g, j, n0, b1[t]);      // rows c*64 + 32t + 8g + i
      xfrag<NS>(xr, p, c * 64 + 32 * t + 4, 2 * g, j, n0, b2[t]);  // rows c*64 + 32t + 8g + 4 + i
    }
    if constexpr (!kFp8) {
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const u32x4 a = *(const u32x4*)(Wb + qv * WB + ((h * 16 + j) * 64 + 32 * t + g * 8) * 2);
#pragma unroll
        for (int s = 0; s < NS; ++s)
          acc[0][s] = Mma<XT>::k32(a, u32x4{b1[t][s].x, b1[t][s].y, b2[t][s].x, b2[t][s].y}, acc[0][s]);
      }
    } else {
      const float sc = p.scales[qv];
      float4_t part[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) part[s] = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const u32x2 codes = *(const u32x2*)(Wb + qv * WB + (h * 16 + j) * 64 + 32 * t + g * 8);
        const u32x2 lo = fp8x4<XT>(codes.x), hi = fp8x4<XT>(codes.y);
        const u32x4 a = {lo.x, lo.y, hi.x, hi.y};
#pragma unroll
        for (int s = 0; s < NS; ++s)
          part[s] = Mma<XT>::k32(a, u32x4{b1[t][s].x, b1[t][s].y, b2[t][s].x, b2[t][s].y}, part[s]);
      }
#pragma unroll
      for (int s = 0; s < NS; ++s) acc[0][s] += sc * part[s];
    }
  }
  row_store<YT, 16, NS>(p, 4 * r + h, n0, lane, acc);  // rows 64r + 16h + 4g + i
}

// The work of one wave in a launch with split rows (light unit).
template <typename XT, typename WT, typename YT, int B, int NS>
__device__ __forceinline__ void row_tile(const RowProblem& p, int32_t r, int32_t n0, int lane) {
  float4_t acc[B / 16][NS];
  row_acc<XT, WT, B, NS>(p, sload(p.row_ptr, r), sload(p.row_ptr, r + 1), n0, lane, acc);
  row_store<YT, B, NS>(p, r, n0, lane, acc);
}

// Row group and column step of light unit lu among rg row groups and ts
// column steps. Default: row groups first. With row slices: the row groups
// in eight balanced slices, each slice's units together (its row groups
// first, then the next column step), so that the contiguous unit range of an
// XCD covers about one slice: the W it streams stays small for every column
// step. Either way a bijection onto (row group, column step).
__device__ __forceinline__ void unit_place(const RowProblem& p, int32_t lu, int32_t rg, int32_t ts, int32_t& g,
                                           int32_t& t) {
  if (!p.row_slices) {
    g = lu % rg;
    t = lu / rg;
    return;
  }
  const int32_t q = rg >> 3, rr = rg & 7;
  const int32_t gi = lu / ts;  // a row group of the slice holding lu
  const int32_t s = gi < rr * (q + 1) ? gi / (q + 1) : rr + (gi - rr * (q + 1)) / max(q, 1);
  const int32_t g0 = s * q + min(s, rr), rows = q + (s < rr ? 1 : 0);
  const int32_t l = lu - g0 * ts;
  g = g0 + l % rows;
  t = l / rows;
}

// Block row r and first column n0 of a wave in light unit lu. Where the
// columns span more than one tile of 16*ns, a unit is two block rows times two
// adjacent column tiles (waves 0, 1 on the first row, 2, 3 on the second): the
// two waves of a row read the same W fragments, close in time, and a unit's
// time is the longer of two rows rather than of four. Otherwise a unit is four
// block rows, one per wave, on the one tile. Consecutive units step through
// the rows first, so the waves resident on an XCD share a few column tiles of
// X (with row slices: one eighth of the rows over every column step, see
// unit_place). With a light-row list the units take its rows in its order
// (the plan lists them longest first and leaves out split rows), else every
// row in order. False: no work for this wave (past the last row or column).
__device__ __forceinline__ bool light_unit(const RowProblem& p, int32_t lu, int wave, int ns, int32_t& r, int32_t& n0) {
  const int32_t tile = 16 * ns;
  const int32_t nl = p.num_light;
  int32_t i, g, t;
  if (p.n > tile) {
    const int32_t rg = (nl + 1) >> 1;
    unit_place(p, lu, rg, (p.n + 2 * tile - 1) / (2 * tile), g, t);
    i = g * 2 + (wave >> 1);
    n0 = (t * 2 + (wave & 1)) * tile;
  } else {
    const int32_t rg = (nl + kRowsPerWg - 1) / kRowsPerWg;
    unit_place(p, lu, rg, (p.n + tile - 1) / tile, g, t);
    i = g * kRowsPerWg + wave;
    n0 = t * tile;
  }
  if (i >= nl || n0 >= p.n) return false;
  r = p.light_rows ? sload(p.light_rows, i) : i;
  return true;
}

// Work units of a problem: heavy units first (one split row or piece times a
// column tile, so the longest units start early), then light units
// (light_unit).
// With pieces and light rows the units are interleaved instead (row_unit).
__device__ __forceinline__ bool interleaved(const RowProblem& p) { return p.part && p.num_light > 0; }
__device__ __forceinline__ int32_t heavy_units(const RowProblem& p, int ns) {
  if (interleaved(p)) return 0;
  return p.num_heavy * ((p.n + 16 * ns - 1) / (16 * ns));
}

// Bytes of LDS a workgroup needs to reduce a split row: three waves' partial
// accumulators (the fourth keeps its own).
__host__ __device__ constexpr int split_lds_bytes(int B, int NS) { return 3 * (B / 16) * NS * 64 * 16; }

// Long rows cut into pieces (Appendix A.2's worst case, all of a partition's
// nonzeros in one row, spread over several workgroups). A piece entry is
// [row, first block, end block, slot, c, C, 0, 0]: piece c of the C pieces of
// its row (C = 1: a whole row, no slot), the row's pieces in consecutive
// slots. A piece of a cut row leaves its FP32 partial for column tile t at
// part[(slot * tiles + t) * 64 NS float4s], in the register layout; the fixup
// kernel (k_piece_fixup), launched next on the same stream, adds a row's
// partials in piece order and stores the row. No workgroup waits for another,
// and the launch boundary makes the partials visible.
template <int NS>
__device__ __forceinline__ void piece_store(const RowProblem& p, int32_t slot, int32_t t, int lane,
                                            const float4_t (&acc)[1][NS]) {
  const int64_t tiles = (p.n + 16 * NS - 1) / (16 * NS);
  float4_t* dst = (float4_t*)p.part + ((int64_t)slot * tiles + t) * (NS * 64);
#pragma unroll
  for (int s = 0; s < NS; ++s) dst[s * 64 + lane] = acc[0][s];
}

// Cut rows of a launch: [num_cut][4] row, first slot, C, 0. One wave per (cut
// row, column tile): Y rows of the block row = the sum of its C partials,
// added in piece order (then the ReLU and the output cast of row_store).
struct FixParams {
  RowProblem pr;
  const int32_t* cut;
  int32_t num_cut;
  int32_t items;  // num_cut x column tiles
};

template <typename YT, int NS>
__global__ __launch_bounds__(256) void k_piece_fixup(FixParams f) {
  const int lane = threadIdx.x & 63;
  const int32_t item = (int32_t)blockIdx.x * 4 + uniform((int32_t)(threadIdx.x >> 6));
  if (item >= f.items) return;
  const RowProblem& p = f.pr;
  const int64_t tiles = (p.n + 16 * NS - 1) / (16 * NS);
  const int32_t cr = item % f.num_cut, t = item / f.num_cut;
  const int32_t r = sload(f.cut, 4 * (int64_t)cr), slot0 = sload(f.cut, 4 * (int64_t)cr + 1);
  const int32_t C = sload(f.cut, 4 * (int64_t)cr + 2);
  const float4_t* __restrict__ part = (const float4_t*)p.part;
  float4_t acc[1][NS];
  const float4_t* src = part + ((int64_t)slot0 * tiles + t) * (NS * 64);
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[0][s] = src[s * 64 + lane];
  for (int32_t c = 1; c < C; ++c) {
    src = part + ((int64_t)(slot0 + c) * tiles + t) * (NS * 64);
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[0][s] += src[s * 64 + lane];
  }
  row_store<YT, 16, NS>(p, r, t * (16 * NS), lane, acc);
}

// One work unit of problem p (local index `unit`). A split row's blocks are cut
// into four pair-aligned ranges, one per wave; waves 1-3 leave their partial
// sums in LDS and wave 0 adds them in wave order, so the result does not depend
// on timing. red: split_lds_bytes(B, NS) of LDS, used only by heavy units.
// SPLIT = false: the problem has no split rows (every unit is light).
template <typename XT, typename WT, typename YT, int B, int NS, bool SPLIT>
__device__ __forceinline__ void row_unit(const RowProblem& p, int32_t unit, int lane, int wave, float4_t* red) {
  constexpr int H = B / 16;
  static_assert(!SPLIT || B == 16, "rows are split for b = 16 only");
  if constexpr (B == 64) {  // a unit is one block row: its four row tiles go to the four waves
    row_tile_b64<XT, WT, YT, NS>(p, unit % p.mb, wave, (unit / p.mb) * (16 * NS), lane);
    return;
  } else if constexpr (!SPLIT) {
    int32_t r, n0;
    if (!light_unit(p, unit, wave, NS, r, n0)) return;
    row_tile_whole<XT, WT, YT, B, NS>(p, r, n0, lane);
    return;
  }
  int32_t e, t;  // split row or piece e, column tile t
  if (interleaved(p)) {
    // Pieces are short: the units go column step by column step (a light
    // unit's tile pair, else its one tile), each step's pieces before its
    // light units, so every XCD works on a few column tiles of X at a time.
    const int32_t tile = 16 * NS, tiles = (p.n + tile - 1) / tile;
    const int32_t tps = p.n > tile ? 2 : 1;
    const int32_t rgl = p.n > tile ? (p.num_light + 1) >> 1 : (p.num_light + kRowsPerWg - 1) / kRowsPerWg;
    const int32_t ph = p.num_heavy * tps, ss = ph + rgl;
    const int32_t step = unit / ss, w = unit - step * ss;
    if (w >= ph) {
      int32_t r, n0;
      if (!light_unit(p, step * rgl + (w - ph), wave, NS, r, n0)) return;
      row_tile<XT, WT, YT, B, NS>(p, r, n0, lane);
      return;
    }
    e = w / tps;
    t = step * tps + (w - e * tps);
    if (t >= tiles) return;  // the second tile of an odd last step
  } else {
    const int32_t hus = heavy_units(p, NS);
    if (unit >= hus) {
      int32_t r, n0;
      if (!light_unit(p, unit - hus, wave, NS, r, n0)) return;
      row_tile<XT, WT, YT, B, NS>(p, r, n0, lane);
      return;
    }
    e = unit % p.num_heavy;
    t = unit / p.num_heavy;
  }
  if constexpr (SPLIT) {
  const int32_t n0 = t * (16 * NS);
  int32_t r, lo, hi, slot = 0, C = 1;
  if (p.part) {  // a piece of a long row, or a whole row
    const int32_t* ent = p.heavy_rows + 8 * (int64_t)e;
    r = sload(ent, 0);
    lo = sload(ent, 1);
    hi = sload(ent, 2);
    slot = sload(ent, 3);
    C = sload(ent, 5);
  } else {
    r = p.heavy_rows ? sload(p.heavy_rows, e) : e;  // no table: every row
    lo = sload(p.row_ptr, r);
    hi = sload(p.row_ptr, r + 1);
  }
  const int32_t seg = (((hi - lo) + 7) / 8) * 2;  // a quarter of the row, rounded up to whole pairs
  const int32_t qa = min(hi, lo + wave * seg), qb = min(hi, qa + seg);
  float4_t acc[H][NS];
  row_acc<XT, WT, B, NS>(p, qa, qb, n0, lane, acc);
  if (wave > 0) {
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
      for (int s = 0; s < NS; ++s) red[(((wave - 1) * H + h) * NS + s) * 64 + lane] = acc[h][s];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
      for (int h = 0; h < H; ++h)
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[h][s] += red[((w * H + h) * NS + s) * 64 + lane];
    if (C > 1) piece_store<NS>(p, slot, t, lane, acc);  // the fixup kernel stores the row
    else row_store<YT, B, NS>(p, r, n0, lane, acc);
  }
  }
}

template <typename XT, typename WT, typename YT, int B, int NS, bool SPLIT>
__global__ __launch_bounds__(256, SPLIT ? 5 : 1) void k_spmm_row(Params prm) {
  if (prm.status && *prm.status) return;
  // (the unsplit form keeps the wave index as a vector value: its row pointer
  // loads then issue as vector loads, which measured faster from cold caches)
  const int lane = threadIdx.x & 63;
  const int wave = SPLIT ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : (int)(threadIdx.x >> 6);
  const RowProblem& p = prm.pr;
  if constexpr (!SPLIT) {
    row_unit<XT, WT, YT, B, NS, false>(p, xcd_unit(blockIdx.x, prm.num_units), lane, wave, nullptr);
  } else {
    // Heavy units take the first workgroups, padded to a multiple of 8; both
    // ranges are numbered so that each XCD runs consecutive units (the same
    // few column tiles of X) and keeps them in its L2.
    extern __shared__ float4_t row_red[];
    const int32_t hus = heavy_units(p, NS);
    const int32_t hpad = (hus + 7) & ~7;
    int32_t unit;
    if ((int32_t)blockIdx.x < hpad) {
      if ((int32_t)blockIdx.x >= hus) return;
      unit = xcd_unit(blockIdx.x, hus);
    } else {
      unit = hus + xcd_unit(blockIdx.x - hpad, prm.num_units - hus);
    }
    row_unit<XT, WT, YT, B, NS, true>(p, unit, lane, wave, row_red);
  }
}

// Whether light units go by row slices (unit_place): from n = 16384, where X
// no longer stays in the Infinity Cache and the W that a pass over a column
// step streams through an XCD's L2 evicts the X slabs between their uses.
// Measured at m = k = 8192, d = 1/16, b = 16, tuned: n = 16384 0.818 against
// 0.930 ms, n = 65536 3.42 against 3.69 ms; n = 8192 no better.
// SPMM_ROW_SLICES=0/1 forces the choice.
inline bool row_slices_preferred(int64_t n) {
  if (const char* e = getenv("SPMM_ROW_SLICES")) return e[0] == '1';
  return n >= 16384;
}

inline RowProblem row_problem(const RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx) {
  RowProblem p{};
  p.row_ptr = row_ptr;
  p.col_idx = col_idx;
  p.W = a.W;
  p.scales = a.scales;
  p.w_index = a.w_index;
  p.X = a.X;
  p.Y = a.Y;
  p.ldx = a.ldx;
  p.ldy = a.ldy;
  p.m = a.plan.m;
  p.k = a.plan.k;
  p.n = a.n;
  p.mb = a.plan.mb;
  p.x_bytes = (uint32_t)((int64_t)a.plan.k * a.ldx * 2);
  p.relu = a.relu ? 1 : 0;
  p.ns = a.ns;
  p.unit_begin = 0;
  p.num_heavy = a.heavy_rows ? a.num_heavy : 0;
  p.heavy_rows = p.num_heavy ? a.heavy_rows : nullptr;
  p.part = p.num_heavy ? a.part : nullptr;
  p.light_rows = a.light_rows;
  p.num_light = a.light_rows ? a.num_light : a.plan.mb;
  p.row_slices = p.num_heavy == 0 && row_slices_preferred(a.n) ? 1 : 0;
  if (a.split_all && a.plan.b == 16) {  // every row split, rows taken in order
    const bool pieces = a.part && a.heavy_rows;  // a table of every row's pieces
    p.num_heavy = pieces ? a.num_heavy : a.plan.mb;
    p.heavy_rows = pieces ? a.heavy_rows : nullptr;
    p.part = pieces ? a.part : nullptr;
    p.light_rows = nullptr;
    p.num_light = 0;
  }
  return p;
}

// Work units of a problem for a column-tile variant: light units over
// num_light rows, heavy units over num_heavy split rows or pieces; inter:
// pieces interleaved with light units, step by step (row_unit).
inline int64_t problem_units(int32_t num_light, int64_t n, int32_t ns, int32_t num_heavy, bool inter) {
  if (inter) {
    const int64_t tile = 16 * ns, tiles = ceil_div(n, tile), tps = n > tile ? 2 : 1;
    const int64_t rgl = n > tile ? ceil_div(num_light, 2) : ceil_div(num_light, kRowsPerWg);
    return ceil_div(tiles, tps) * (num_heavy * tps + rgl);
  }
  const int64_t light = n > 16 * ns ? ceil_div(num_light, 2) * ceil_div(n, 32 * ns)
                                    : ceil_div(num_light, kRowsPerWg) * ceil_div(n, 16 * ns);
  return light + (int64_t)num_heavy * ceil_div(n, 16 * ns);
}

// The fixup launch of the cut rows of a problem whose pieces ran with tile
// width ns (the same as its main launch).
template <typename YT>
spmm_status_t launch_piece_fixup(const RowProblem& pr, const int32_t* cut_rows, int32_t num_cut, int ns,
                                 hipStream_t stream) {
  FixParams f;
  f.pr = pr;
  f.cut = cut_rows;
  f.num_cut = num_cut;
  const int64_t items = (int64_t)num_cut * ceil_div(pr.n, 16 * ns);
  if (items == 0) return SPMM_OK;
  if (items > (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "too many work units");
  f.items = (int32_t)items;
  const dim3 grid((unsigned)ceil_div(items, 4));
  if (ns == 8) hipLaunchKernelGGL((k_piece_fixup<YT, 8>), grid, dim3(256), 0, stream, f);
  else if (ns == 4) hipLaunchKernelGGL((k_piece_fixup<YT, 4>), grid, dim3(256), 0, stream, f);
  else if (ns == 2) hipLaunchKernelGGL((k_piece_fixup<YT, 2>), grid, dim3(256), 0, stream, f);
  else return fail(SPMM_ERR_INVALID_ARG, "column tile variant must be 2, 4 or 8");
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

template <typename XT, typename WT, typename YT, int B>
spmm_status_t launch_row(const RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx, hipStream_t stream) {
  if ((int64_t)a.plan.k * a.ldx * 2 >= (int64_t)INT32_MAX)
    return fail(SPMM_ERR_UNSUPPORTED, "X larger than 2 GiB is not supported");
  Params prm;
  prm.pr = row_problem(a, row_ptr, col_idx);
  prm.status = a.status;
  const int ns = prm.pr.ns;
  const int64_t units = B == 64 ? (int64_t)a.plan.mb * ceil_div(a.n, 16 * ns)
                                : problem_units(prm.pr.num_light, a.n, ns, prm.pr.num_heavy,
                                                prm.pr.part && prm.pr.num_light > 0);
  if (units == 0) return SPMM_OK;
  if (units > (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "too many work units");
  prm.num_units = (int32_t)units;
  const bool inter = prm.pr.part && prm.pr.num_light > 0;
  const int64_t hus = B == 16 && !inter ? (int64_t)prm.pr.num_heavy * ceil_div(a.n, 16 * ns) : 0;
  const int64_t grid = units + (((hus + 7) & ~(int64_t)7) - hus);
  if (grid > (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "too many work units");
  const bool split = B == 16 && prm.pr.num_heavy > 0;
  const unsigned lds = split ? (unsigned)split_lds_bytes(B, ns) : 0u;
  if (split) {
    if constexpr (B == 16) {
      if (ns == 8) hipLaunchKernelGGL((k_spmm_row<XT, WT, YT, B, 8, true>), dim3((unsigned)grid), dim3(256), lds, stream, prm);
      else if (ns == 4) hipLaunchKernelGGL((k_spmm_row<XT, WT, YT, B, 4, true>), dim3((unsigned)grid), dim3(256), lds, stream, prm);
      else if (ns == 2) hipLaunchKernelGGL((k_spmm_row<XT, WT, YT, B, 2, true>), dim3((unsigned)grid), dim3(256), lds, stream, prm);
      else return fail(SPMM_ERR_INVALID_ARG, "column tile variant must be 2, 4 or 8");
    }
  }
  else if (ns == 8) hipLaunchKernelGGL((k_spmm_row<XT, WT, YT, B, 8, false>), dim3((unsigned)grid), dim3(256), 0, stream, prm);
  else if (ns == 4) hipLaunchKernelGGL((k_spmm_row<XT, WT, YT, B, 4, false>), dim3((unsigned)grid), dim3(256), 0, stream, prm);
  else if (ns == 2) hipLaunchKernelGGL((k_spmm_row<XT, WT, YT, B, 2, false>), dim3((unsigned)grid), dim3(256), 0, stream, prm);
  else return fail(SPMM_ERR_INVALID_ARG, "column tile variant must be 2, 4 or 8");
  SPMM_HIP(hipGetLastError());
  if constexpr (B == 16) {
    if (prm.pr.part && a.num_cut > 0) return launch_piece_fixup<YT>(prm.pr, a.cut_rows, a.num_cut, ns, stream);
  }
  return SPMM_OK;
}

}  // namespace row
}  // namespace spmm
