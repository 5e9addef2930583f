// Block-sparse x dense SpMM for the small block sizes 1, 4 and 8, on the
// vector ALUs (PopSparse, Section 3: Y = (M o W) * X with FP32 accumulation;
// the paper's b = 1 case is unstructured sparsity).
//
// A b x b block with b < 16 fills a 16-wide matrix-core tile only partly, so
// these sizes run on VALU dot products instead. One wave owns one block row
// and a tile of 64*V columns: lane j covers V consecutive columns and keeps
// b x V FP32 accumulators. The wave walks the row's blocks in block-CSR order:
//   * the block's weights are uniform across the wave (scalar loads for
//     b = 4/8; for b = 1 a chunk of 64 weights and columns is loaded one per
//     lane and broadcast with v_readlane);
//   * the lane loads V elements (8 or 16 bytes) of each of the block's b X
//     rows with buffer loads, which return zero past the end of X (k tail).
// With 16-bit X and weights the inner product runs on v_dot2 (two products
// per instruction, FP32 accumulate): for b = 4/8 the pair is two consecutive k
// values of one block, interleaved from two X rows with v_perm; for b = 1 the
// pair is two consecutive nonzeros of the row. FP32 and FP8 weights take FP32
// FMAs (an FP8 weight is decoded exactly and multiplied by its block scale).
// Workgroups are ordered XCD-aware, as in the row-wise MFMA kernel.
#include <cstdlib>

#include "common.h"

namespace spmm {
namespace {

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

struct Fp8 {};  // weights stored as OCP E4M3FN codes

struct SParams {
  const int32_t* row_ptr;  // [mb + 1]
  const int32_t* col_idx;  // [nnz]
  const void* W;           // values in block-CSR order (or indexed by w_index), row-major b x b per block
  const float* scales;     // FP8 block scales, indexed like W, else nullptr
  const int32_t* w_index;  // entry q's values are block w_index[q] of W; nullptr: block q
  const void* X;
  void* Y;
  int64_t ldx, ldy;
  int32_t m, k, n, mb;
  int32_t num_units;
  uint32_t x_bytes;        // k * ldx * sizeof(X element), < 2^31
  int32_t relu;            // nonzero: max(0, y) before the output cast
  const int32_t* status;   // skip when *status != 0 (dynamic), else nullptr
  int32_t row_slices;      // S > 0: units ordered by S slices of the row groups (unit_place)
};

constexpr uint32_t kOOB = 0x80000000u;
constexpr int kRowsPerWg = 4;  // one block row per wave

__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int32_t xcd_unit(int32_t w, int32_t U) {
  const int32_t q = U >> 3, r = U & 7;
  const int32_t x = w & 7, local = w >> 3;
  return x * q + min(x, r) + local;
}

// Row group g and column tile t of unit u among rg row groups and ts tiles:
// row groups first, or, with S row slices, the row groups in S balanced
// slices whose units come together (row groups first within a slice), so
// that an XCD's contiguous eighth of the units reads an S-th of the indices
// and weights for every column tile. A bijection either way.
__device__ __forceinline__ void unit_place(int32_t u, int32_t rg, int32_t ts, int32_t S, int32_t& g, int32_t& t) {
  if (S == 0) {
    g = u % rg;
    t = u / rg;
    return;
  }
  const int32_t q = rg / S, rr = rg - q * S;
  const int32_t gi = u / ts;  // a row group of the slice holding u
  const int32_t s = gi < rr * (q + 1) ? gi / (q + 1) : rr + (gi - rr * (q + 1)) / max(q, 1);
  const int32_t g0 = s * q + min(s, rr), rows = q + (s < rr ? 1 : 0);
  const int32_t l = u - g0 * ts;
  g = g0 + l % rows;
  t = l / rows;
}

template <typename T> struct Num;
template <> struct Num<_Float16> {
  static __device__ __forceinline__ float dot2(uint32_t a, uint32_t b, float c) {
    return __builtin_amdgcn_fdot2(__builtin_bit_cast(half2_t, a), __builtin_bit_cast(half2_t, b), c, false);
  }
  static __device__ __forceinline__ float lo(uint32_t v) { return (float)__builtin_bit_cast(_Float16, (uint16_t)v); }
  static __device__ __forceinline__ float hi(uint32_t v) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(v >> 16));
  }
  static __device__ __forceinline__ uint16_t store(float v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
};
template <> struct Num<__bf16> {
  static __device__ __forceinline__ float dot2(uint32_t a, uint32_t b, float c) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a), __builtin_bit_cast(bf16x2_t, b), c, false);
  }
  static __device__ __forceinline__ float lo(uint32_t v) { return __builtin_bit_cast(float, v << 16); }
  static __device__ __forceinline__ float hi(uint32_t v) { return __builtin_bit_cast(float, v & 0xFFFF0000u); }
  static __device__ __forceinline__ uint16_t store(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
};

// V elements of one X row (k row `krow`, columns col0 .. col0 + V) as dwords.
template <typename XT, int V>
struct XRow {
  static constexpr int BYTES = V * (int)sizeof(XT);
  static constexpr int DW = BYTES / 4;
  static_assert(BYTES == 8 || BYTES == 16, "8- or 16-byte loads per lane");
  static __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t xr, uint32_t off, uint32_t (&d)[DW]) {
    if constexpr (BYTES == 16) {
      const u32x4 v = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(xr, off, 0, 0));
#pragma unroll
      for (int i = 0; i < 4; ++i) d[i] = v[i];
    } else {
      const u32x2 v = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(xr, off, 0, 0));
      d[0] = v.x;
      d[1] = v.y;
    }
  }
};

// Element v of a row held as dwords, as float.
template <typename XT, int DW>
__device__ __forceinline__ float x_elem(const uint32_t (&d)[DW], int v) {
  if constexpr (sizeof(XT) == 4) return __builtin_bit_cast(float, d[v]);
  else return (v & 1) ? Num<XT>::hi(d[v >> 1]) : Num<XT>::lo(d[v >> 1]);
}

// One weight as float: 16-bit and FP32 weights directly, FP8 decoded and scaled.
template <typename XT, typename WT>
__device__ __forceinline__ float w_elem(const uint8_t* __restrict__ Wb, int64_t idx, float scale) {
  if constexpr (__is_same(WT, Fp8)) {
    const uint32_t code = Wb[idx];
    return __builtin_amdgcn_cvt_f32_fp8((int)code, 0) * scale;
  } else if constexpr (sizeof(WT) == 4) {
    return ((const float*)Wb)[idx];
  } else {
    const uint32_t h = ((const uint16_t*)Wb)[idx];
    return Num<WT>::lo(h);
  }
}

template <typename XT, typename WT, typename YT, int B, int V>
__global__ __launch_bounds__(256) void k_spmm_small(SParams p) {
  if (p.status && *p.status) return;
  using XR = XRow<XT, V>;
  constexpr int DW = XR::DW;
  constexpr int XE = sizeof(XT);
  constexpr bool kDot = sizeof(XT) == 2 && __is_same(XT, WT);  // 16-bit weights and X
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int32_t unit = xcd_unit(blockIdx.x, p.num_units);
  const int32_t rgroups = (p.mb + kRowsPerWg - 1) / kRowsPerWg;
  int32_t rg, ct;
  unit_place(unit, rgroups, (p.n + 64 * V - 1) / (64 * V), p.row_slices, rg, ct);
  const int32_t n0 = ct * (64 * V);
  const int32_t r = rg * kRowsPerWg + wave;
  if (r >= p.mb) return;
  const int32_t col0 = n0 + V * lane;
  const uint32_t lane_off = (uint32_t)(col0 * XE);

  __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)p.X, (short)0, (int)p.x_bytes, 0x00020000);
  const uint8_t* __restrict__ Wb = (const uint8_t*)p.W;
  float acc[B][V];
#pragma unroll
  for (int i = 0; i < B; ++i)
#pragma unroll
    for (int v = 0; v < V; ++v) acc[i][v] = 0.f;

  const int32_t q_lo = uniform(p.row_ptr[r]), q_hi = uniform(p.row_ptr[r + 1]);
  auto xoff = [&](int32_t krow) -> uint32_t {
    return (krow >= 0 && krow < p.k) ? (uint32_t)((int64_t)krow * p.ldx * XE) + lane_off : kOOB;
  };

  if constexpr (B == 1) {
    // chunks of 64 nonzeros: lane t holds the column and weight of entry q0 + t
    for (int32_t q0 = q_lo; q0 < q_hi; q0 += 64) {
      const int32_t cnt = min(64, q_hi - q0);
      const bool have = lane < cnt;
      const int32_t cv = have ? p.col_idx[q0 + lane] : -1;
      uint32_t wv = 0;  // 16-bit weight bits, or float bits
      if (have) {
        const int32_t qi = p.w_index ? p.w_index[q0 + lane] : q0 + lane;
        if constexpr (kDot) wv = ((const uint16_t*)Wb)[qi];
        else wv = __builtin_bit_cast(uint32_t, w_elem<XT, WT>(Wb, qi, __is_same(WT, Fp8) ? p.scales[qi] : 1.f));
      }
      for (int32_t t = 0; t < cnt; t += 8) {
        uint32_t xd[8][DW];
        int32_t c[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          // slots past the chunk read nothing (zero loads) and weigh zero
          c[u] = t + u < cnt ? __builtin_amdgcn_readlane(cv, (t + u) & 63) : -1;
          XR::load(xr, xoff(c[u]), xd[u]);
        }
        if constexpr (kDot) {
#pragma unroll
          for (int u = 0; u < 8; u += 2) {
            const uint32_t w1 = t + u < cnt ? __builtin_amdgcn_readlane(wv, (t + u) & 63) : 0u;
            const uint32_t w2 = t + u + 1 < cnt ? __builtin_amdgcn_readlane(wv, (t + u + 1) & 63) : 0u;
            const uint32_t wp = (w1 & 0xFFFFu) | (w2 << 16);
#pragma unroll
            for (int v = 0; v < V; ++v) {
              const uint32_t sel = (v & 1) ? 0x07060302u : 0x05040100u;
              const uint32_t xp = __builtin_amdgcn_perm(xd[u + 1][v >> 1], xd[u][v >> 1], sel);
              acc[0][v] = Num<XT>::dot2(wp, xp, acc[0][v]);
            }
          }
        } else {
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const float w = t + u < cnt ? __builtin_bit_cast(float, __builtin_amdgcn_readlane(wv, (t + u) & 63)) : 0.f;
#pragma unroll
            for (int v = 0; v < V; ++v) acc[0][v] = __builtin_fmaf(w, x_elem<XT, DW>(xd[u], v), acc[0][v]);
          }
        }
      }
    }
  } else if constexpr (kDot) {
    // b = 4 / 8: weights as dword pairs along k (row-major block), X rows
    // interleaved pairwise into (k, k + 1) dwords
    constexpr int WD = B * B / 2;  // dwords per block
    for (int32_t q = q_lo; q < q_hi; ++q) {
      const int32_t c = uniform(p.col_idx[q]);
      const int64_t qv = p.w_index ? (int64_t)uniform(p.w_index[q]) : (int64_t)q;
      const uint32_t* __restrict__ wq = (const uint32_t*)(Wb + qv * B * B * 2);
      uint32_t wd[WD];
#pragma unroll
      for (int i = 0; i < WD; ++i) wd[i] = wq[i];
      uint32_t xd[B][DW];
#pragma unroll
      for (int kk = 0; kk < B; ++kk) XR::load(xr, xoff(c * B + kk), xd[kk]);
#pragma unroll
      for (int kp = 0; kp < B / 2; ++kp) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const uint32_t sel = (v & 1) ? 0x07060302u : 0x05040100u;
          const uint32_t xp = __builtin_amdgcn_perm(xd[2 * kp + 1][v >> 1], xd[2 * kp][v >> 1], sel);
#pragma unroll
          for (int i = 0; i < B; ++i) acc[i][v] = Num<XT>::dot2(wd[i * (B / 2) + kp], xp, acc[i][v]);
        }
      }
    }
  } else {
    // FP32 or FP8 weights: FP32 FMAs
    for (int32_t q = q_lo; q < q_hi; ++q) {
      const int32_t c = uniform(p.col_idx[q]);
      const int64_t qv = p.w_index ? (int64_t)uniform(p.w_index[q]) : (int64_t)q;
      const float sc = __is_same(WT, Fp8) ? p.scales[qv] : 1.f;
      float w[B][B];
#pragma unroll
      for (int i = 0; i < B; ++i)
#pragma unroll
        for (int kk = 0; kk < B; ++kk) w[i][kk] = w_elem<XT, WT>(Wb, qv * B * B + i * B + kk, sc);
#pragma unroll
      for (int kk = 0; kk < B; ++kk) {
        uint32_t xd[DW];
        XR::load(xr, xoff(c * B + kk), xd);
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const float x = x_elem<XT, DW>(xd, v);
#pragma unroll
          for (int i = 0; i < B; ++i) acc[i][v] = __builtin_fmaf(w[i][kk], x, acc[i][v]);
        }
      }
    }
  }

  // epilogue: lane holds rows r*B + i and columns col0 .. col0 + V
  if (p.relu) {
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
      for (int v = 0; v < V; ++v) acc[i][v] = acc[i][v] > 0.f ? acc[i][v] : 0.f;
  }
  YT* __restrict__ Y = (YT*)p.Y;
#pragma unroll
  for (int i = 0; i < B; ++i) {
    const int64_t row = (int64_t)r * B + i;
    if (row >= p.m) continue;
    YT* dst = Y + row * p.ldy + col0;
    if (col0 + V <= p.n) {
      if constexpr (sizeof(YT) == 4) {
#pragma unroll
        for (int v = 0; v < V; v += 4)
          *(float4_t*)(dst + v) = float4_t{acc[i][v], acc[i][v + 1], acc[i][v + 2], acc[i][v + 3]};
      } else {
        uint32_t o[V / 2];
#pragma unroll
        for (int e = 0; e < V / 2; ++e)
          o[e] = (uint32_t)Num<YT>::store(acc[i][2 * e]) | ((uint32_t)Num<YT>::store(acc[i][2 * e + 1]) << 16);
        if constexpr (V == 8) *(u32x4*)dst = u32x4{o[0], o[1], o[2], o[3]};
        else *(u32x2*)dst = u32x2{o[0], o[1]};
      }
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v)
        if (col0 + v < p.n) {
          if constexpr (sizeof(YT) == 4) dst[v] = acc[i][v];
          else ((uint16_t*)dst)[v] = Num<YT>::store(acc[i][v]);
        }
    }
  }
}

// ------------------------------------------------------------------ b = 4 / 8 on MFMA
// With 16-bit weights and X, b = 4 and 8 run on 16x16x32 MFMAs: 32 / b blocks
// of one block row fill the 32 k slots of one instruction (lane group g takes
// 8 / b of them), the block row's b rows occupy the first b of the 16 A rows
// (the rest are zero). Per lane group the B operand is 8 X rows (the k rows of
// its blocks) x 8 columns, loaded as 16-byte rows and transposed with v_perm,
// so that MFMA tile s covers physical columns 8j + s as in the row-wise
// kernel. Half (b = 8) or a quarter (b = 4) of each MFMA is useful work, which
// still leaves the matrix cores far from being the limit: these block sizes
// are bound by the X reads (b FLOPs per byte from L2).
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

template <typename XT> struct Mfma;
template <> struct Mfma<_Float16> {
  static __device__ __forceinline__ float4_t k32(u32x4 a, u32x4 b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(half8_t, a), __builtin_bit_cast(half8_t, b), c, 0, 0, 0);
  }
};
template <> struct Mfma<__bf16> {
  static __device__ __forceinline__ float4_t k32(u32x4 a, u32x4 b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c, 0, 0, 0);
  }
};

template <typename XT, typename YT, int B>
__global__ __launch_bounds__(256) void k_spmm_small_mfma(SParams p) {
  static_assert(B == 4 || B == 8, "MFMA form of the small block sizes");
  constexpr int BPM = 32 / B;  // blocks per MFMA
  constexpr int BPG = 8 / B;   // blocks per lane group
  if (p.status && *p.status) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  const int32_t unit = xcd_unit(blockIdx.x, p.num_units);
  const int32_t rgroups = (p.mb + kRowsPerWg - 1) / kRowsPerWg;
  int32_t rgi, ct;
  unit_place(unit, rgroups, (p.n + 127) / 128, p.row_slices, rgi, ct);
  const int32_t r = rgi * kRowsPerWg + wave;
  const int32_t n0 = ct * 128;
  if (r >= p.mb) return;
  __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)p.X, (short)0, (int)p.x_bytes, 0x00020000);
  const uint8_t* __restrict__ Wb = (const uint8_t*)p.W;
  const uint32_t lane_off = (uint32_t)((n0 + 8 * j) * 2);
  float4_t acc[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) acc[s] = float4_t{0.f, 0.f, 0.f, 0.f};
  const int32_t q_lo = uniform(p.row_ptr[r]), q_hi = uniform(p.row_ptr[r + 1]);
  for (int32_t q = q_lo; q < q_hi; q += BPM) {
    // this lane group's blocks: q + g*BPG + t
    uint32_t adw[4] = {0u, 0u, 0u, 0u};
    uint32_t rows[8][4];
#pragma unroll
    for (int t = 0; t < BPG; ++t) {
      const int32_t qb = q + g * BPG + t;
      const bool ok = qb < q_hi;
      const int32_t c = ok ? p.col_idx[qb] : 0;
      const int64_t qv = ok ? (p.w_index ? (int64_t)p.w_index[qb] : (int64_t)qb) : 0;
      if (ok && j < B) {
        // row j of block qb: B 16-bit weights
        const uint8_t* src = Wb + qv * (B * B * 2) + j * (B * 2);
        if constexpr (B == 8) {
          const u32x4 w = *(const u32x4*)src;
          adw[0] = w[0]; adw[1] = w[1]; adw[2] = w[2]; adw[3] = w[3];
        } else {
          const u32x2 w = *(const u32x2*)src;
          adw[2 * t] = w.x;
          adw[2 * t + 1] = w.y;
        }
      }
#pragma unroll
      for (int e = 0; e < B; ++e) {
        const int32_t krow = c * B + e;
        const uint32_t off = (ok && krow < p.k) ? (uint32_t)((int64_t)krow * p.ldx * 2) + lane_off : kOOB;
        const u32x4 v = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(xr, off, 0, 0));
#pragma unroll
        for (int d = 0; d < 4; ++d) rows[t * B + e][d] = v[d];
      }
    }
    const u32x4 a = {adw[0], adw[1], adw[2], adw[3]};
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const uint32_t sel = (s & 1) ? 0x07060302u : 0x05040100u;
      u32x4 bv;
#pragma unroll
      for (int d = 0; d < 4; ++d) bv[d] = __builtin_amdgcn_perm(rows[2 * d + 1][s >> 1], rows[2 * d][s >> 1], sel);
      acc[s] = Mfma<XT>::k32(a, bv, acc[s]);
    }
  }
  // epilogue: lane (g, j) holds rows 4g + i (valid below B), columns n0 + 8j .. +8
  if (4 * g >= B) return;
  if (p.relu) {
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[s][i] = acc[s][i] > 0.f ? acc[s][i] : 0.f;
  }
  YT* __restrict__ Y = (YT*)p.Y;
  const int32_t col0 = n0 + 8 * j;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = (int64_t)r * B + 4 * g + i;
    if (row >= p.m) continue;
    YT* dst = Y + row * p.ldy + col0;
    if (col0 + 8 <= p.n) {
      if constexpr (sizeof(YT) == 4) {
        *(float4_t*)dst = float4_t{acc[0][i], acc[1][i], acc[2][i], acc[3][i]};
        *(float4_t*)(dst + 4) = float4_t{acc[4][i], acc[5][i], acc[6][i], acc[7][i]};
      } else {
        uint32_t o[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
          o[e] = (uint32_t)Num<YT>::store(acc[2 * e][i]) | ((uint32_t)Num<YT>::store(acc[2 * e + 1][i]) << 16);
        *(u32x4*)dst = u32x4{o[0], o[1], o[2], o[3]};
      }
    } else {
#pragma unroll
      for (int s = 0; s < 8; ++s)
        if (col0 + s < p.n) {
          if constexpr (sizeof(YT) == 4) dst[s] = acc[s][i];
          else ((uint16_t*)dst)[s] = Num<YT>::store(acc[s][i]);
        }
    }
  }
}

// The same computation with its block loop software-pipelined, for launches
// with few workgroups per CU, where nothing else hides the loads' latency:
// the next group of blocks is loaded into a second buffer while the current
// group's MFMAs run. As in the pipelined row-wise kernel, every load is
// unconditional (indices clamped, X offsets out of range past the row's end,
// weight rows clamped and masked at MFMA time), the X rows are transposed only
// at MFMA time, and the column and value indices of up to 64 blocks come from
// one vector load, handed to each lane group with a lane permute. Chunks of 64
// blocks start at multiples of 32 / b blocks from the row's start, so the
// groups, and the MFMA inputs, are those of the plain kernel: the results are
// the same bit for bit.
template <int B>
struct SmallBuf {
  uint32_t adw[4];     // A operand: row j of this lane group's blocks (unmasked)
  uint32_t rows[8][4]; // raw X rows of this lane group's blocks
};

template <typename XT, typename YT, int B>
__global__ __launch_bounds__(256) void k_spmm_small_mfma_pp(SParams p) {
  static_assert(B == 4 || B == 8, "MFMA form of the small block sizes");
  constexpr int BPM = 32 / B;  // blocks per MFMA
  constexpr int BPG = 8 / B;   // blocks per lane group
  if (p.status && *p.status) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  const int32_t unit = xcd_unit(blockIdx.x, p.num_units);
  const int32_t rgroups = (p.mb + kRowsPerWg - 1) / kRowsPerWg;
  int32_t rgi, ct;
  unit_place(unit, rgroups, (p.n + 127) / 128, p.row_slices, rgi, ct);
  const int32_t r = rgi * kRowsPerWg + wave;
  const int32_t n0 = ct * 128;
  if (r >= p.mb) return;
  __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)p.X, (short)0, (int)p.x_bytes, 0x00020000);
  const uint8_t* __restrict__ Wb = (const uint8_t*)p.W;
  const uint32_t lane_off = (uint32_t)((n0 + 8 * j) * 2);
  const int jj = j < B ? j : B - 1;  // weight row read by this lane (rows j >= B are masked)
  float4_t acc[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) acc[s] = float4_t{0.f, 0.f, 0.f, 0.f};
  const int32_t q_lo = uniform(p.row_ptr[r]), q_hi = uniform(p.row_ptr[r + 1]);
  for (int32_t c0 = q_lo; c0 < q_hi; c0 += 64) {
    const int32_t cn = min(64, q_hi - c0);
    const int32_t civ = lane < cn ? p.col_idx[c0 + lane] : 0;
    const int32_t wiv = p.w_index ? (lane < cn ? p.w_index[c0 + lane] : 0) : c0 + lane;
    // the group of BPM blocks starting at chunk offset t; lane group g takes BPG of them
    auto load = [&](int32_t t, SmallBuf<B>& S) {
#pragma unroll
      for (int tt = 0; tt < BPG; ++tt) {
        const int32_t idx = t + g * BPG + tt;
        const int32_t ic = min(idx, cn - 1);
        const int32_t c = __shfl(civ, ic, 64);
        const int64_t qv = __shfl(wiv, ic, 64);
        const uint8_t* src = Wb + qv * (B * B * 2) + jj * (B * 2);
        if constexpr (B == 8) {
          const u32x4 w = *(const u32x4*)src;
          S.adw[0] = w[0]; S.adw[1] = w[1]; S.adw[2] = w[2]; S.adw[3] = w[3];
        } else {
          const u32x2 w = *(const u32x2*)src;
          S.adw[2 * tt] = w.x;
          S.adw[2 * tt + 1] = w.y;
        }
#pragma unroll
        for (int e = 0; e < B; ++e) {
          const int32_t krow = c * B + e;
          const uint32_t off = (idx < cn && krow < p.k) ? (uint32_t)((int64_t)krow * p.ldx * 2) + lane_off : kOOB;
          const u32x4 v = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(xr, off, 0, 0));
#pragma unroll
          for (int d = 0; d < 4; ++d) S.rows[tt * B + e][d] = v[d];
        }
      }
    };
    auto mma = [&](int32_t t, const SmallBuf<B>& S) {
      // A: zero for lanes j >= B and for blocks past the row's end, as in the plain kernel
      u32x4 a;
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const int tt = B == 8 ? 0 : d / 2;
        a[d] = (j < B && t + g * BPG + tt < cn) ? S.adw[d] : 0u;
      }
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const uint32_t sel = (s & 1) ? 0x07060302u : 0x05040100u;
        u32x4 bv;
#pragma unroll
        for (int d = 0; d < 4; ++d) bv[d] = __builtin_amdgcn_perm(S.rows[2 * d + 1][s >> 1], S.rows[2 * d][s >> 1], sel);
        acc[s] = Mfma<XT>::k32(a, bv, acc[s]);
      }
    };
    SmallBuf<B> A, Bf;
    load(0, A);
    for (int32_t t = 0; t < cn; t += 2 * BPM) {
      load(t + BPM, Bf);
      mma(t, A);
      if (t + BPM >= cn) break;
      load(t + 2 * BPM, A);
      mma(t + BPM, Bf);
    }
  }
  // epilogue: as in the plain kernel
  if (4 * g >= B) return;
  if (p.relu) {
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[s][i] = acc[s][i] > 0.f ? acc[s][i] : 0.f;
  }
  YT* __restrict__ Y = (YT*)p.Y;
  const int32_t col0 = n0 + 8 * j;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = (int64_t)r * B + 4 * g + i;
    if (row >= p.m) continue;
    YT* dst = Y + row * p.ldy + col0;
    if (col0 + 8 <= p.n) {
      if constexpr (sizeof(YT) == 4) {
        *(float4_t*)dst = float4_t{acc[0][i], acc[1][i], acc[2][i], acc[3][i]};
        *(float4_t*)(dst + 4) = float4_t{acc[4][i], acc[5][i], acc[6][i], acc[7][i]};
      } else {
        uint32_t o[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
          o[e] = (uint32_t)Num<YT>::store(acc[2 * e][i]) | ((uint32_t)Num<YT>::store(acc[2 * e + 1][i]) << 16);
        *(u32x4*)dst = u32x4{o[0], o[1], o[2], o[3]};
      }
    } else {
#pragma unroll
      for (int s = 0; s < 8; ++s)
        if (col0 + s < p.n) {
          if constexpr (sizeof(YT) == 4) dst[s] = acc[s][i];
          else ((uint16_t*)dst)[s] = Num<YT>::store(acc[s][i]);
        }
    }
  }
}

// The pipelined MFMA form for launches of at most eight workgroups per CU
// whose rows average at least four groups of 32 / b blocks. Measured at
// m = k = 8192: n = 256, b = 8 (512 workgroups) 11 - 22% faster, b = 4 (1024)
// 13%, n = 1024, b = 8 (2048) 6%; one loss, m = k = 2048, n = 1024, b = 4
// (1024 workgroups, rows of 64 blocks), 5% slower. SPMM_SMALL_PP=0/1 forces
// the choice (for comparisons).
bool small_pp_preferred(int32_t b, int64_t units, int32_t mb, int64_t nnz, int num_cus) {
  if (const char* e = getenv("SPMM_SMALL_PP")) return e[0] == '1';
  return units <= 8 * (int64_t)num_cus && nnz >= 4 * (32 / b) * (int64_t)mb;
}

// Row slices of the units (unit_place), 0 for none: eight where X no longer
// stays in the Infinity Cache and the indices and weights that a pass over a
// column tile streams through an XCD's L2 evict X between its uses. Measured
// at m = k = 8192 (FP16, the kernel without LDS), eight slices against none:
// n = 16384, b = 8 1.22 against 1.70 ms at d = 1/16, b = 4 1.44 against 1.73
// ms at 1/32, b = 1 6.13 against 6.70 ms at 1/32; n = 8192, d = 1/16, b = 8
// 0.486 against 0.601 ms, b = 4 1.15 against 1.25 ms, but b = 1 4.63
// against 4.35 ms; n <= 4096 no better at any block size. SPMM_SMALL_SLICES
// =0/2/4/8 forces the count.
int32_t small_row_slices(int64_t n, int32_t b) {
  if (const char* e = getenv("SPMM_SMALL_SLICES")) {
    const int v = atoi(e);
    return (v == 2 || v == 4 || v == 8) ? v : 0;
  }
  return n >= (b == 1 ? 16384 : 8192) ? 8 : 0;
}

template <typename XT, typename WT, typename YT, int B, int V>
spmm_status_t launch_small(const RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx, hipStream_t s) {
  SParams p;
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
  p.status = a.status;
  p.relu = a.relu ? 1 : 0;
  p.row_slices = small_row_slices(a.n, B);
  const int64_t xb = (int64_t)a.plan.k * a.ldx * (int64_t)sizeof(XT);
  if (xb >= (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "X larger than 2 GiB is not supported");
  p.x_bytes = (uint32_t)xb;
  constexpr bool kMfma = (B == 4 || B == 8) && sizeof(XT) == 2 && __is_same(XT, WT);
  const int64_t tile = kMfma ? 128 : 64 * V;
  const int64_t units = ceil_div(a.plan.mb, kRowsPerWg) * ceil_div(a.n, tile);
  if (units == 0) return SPMM_OK;
  if (units > (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "too many work units");
  p.num_units = (int32_t)units;
  if constexpr (kMfma) {
    if (small_pp_preferred(B, units, a.plan.mb, a.nnz, device_cu_count()))
      hipLaunchKernelGGL((k_spmm_small_mfma_pp<XT, YT, B>), dim3((unsigned)units), dim3(256), 0, s, p);
    else
      hipLaunchKernelGGL((k_spmm_small_mfma<XT, YT, B>), dim3((unsigned)units), dim3(256), 0, s, p);
  }
  else
    hipLaunchKernelGGL((k_spmm_small<XT, WT, YT, B, V>), dim3((unsigned)units), dim3(256), 0, s, p);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

// columns per lane: the requested variant (4 or 8), else 8 (16-byte loads of
// 16-bit X) unless n is small enough that a 256-column tile already covers it
template <typename XT, typename WT, typename YT, int B>
spmm_status_t small_v(const RunArgs& a, const int32_t* rp, const int32_t* ci, hipStream_t s) {
  if constexpr (sizeof(XT) == 4) return launch_small<XT, WT, YT, B, 4>(a, rp, ci, s);
  else if constexpr ((B == 4 || B == 8) && __is_same(XT, WT)) return launch_small<XT, WT, YT, B, 8>(a, rp, ci, s);
  else {
    const int v = (a.ns == 4 || a.ns == 8) ? a.ns : (a.n <= 256 ? 4 : 8);
    if (v == 4) return launch_small<XT, WT, YT, B, 4>(a, rp, ci, s);
    return launch_small<XT, WT, YT, B, 8>(a, rp, ci, s);
  }
}

template <typename XT, typename WT, typename YT>
spmm_status_t small_b(const RunArgs& a, const int32_t* rp, const int32_t* ci, hipStream_t s) {
  switch (a.plan.b) {
    case 1: return small_v<XT, WT, YT, 1>(a, rp, ci, s);
    case 4: return small_v<XT, WT, YT, 4>(a, rp, ci, s);
    case 8: return small_v<XT, WT, YT, 8>(a, rp, ci, s);
  }
  return fail(SPMM_ERR_UNSUPPORTED, "small-block kernel handles block sizes 1, 4 and 8");
}

template <typename XT, typename WT>
spmm_status_t small_y(const RunArgs& a, const int32_t* rp, const int32_t* ci, hipStream_t s) {
  if (a.yt == SPMM_F32) return small_b<XT, WT, float>(a, rp, ci, s);
  return small_b<XT, WT, XT>(a, rp, ci, s);
}

}  // namespace

spmm_status_t launch_spmm_small(const RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx, hipStream_t s) {
  using bf = __bf16;
  if (a.wt == SPMM_F32) return small_y<float, float>(a, row_ptr, col_idx, s);
  if (a.wt == SPMM_FP8_E4M3) {
    if (a.xt == SPMM_F16) return small_y<_Float16, Fp8>(a, row_ptr, col_idx, s);
    return small_y<bf, Fp8>(a, row_ptr, col_idx, s);
  }
  if (a.wt == SPMM_F16) return small_y<_Float16, _Float16>(a, row_ptr, col_idx, s);
  return small_y<bf, bf>(a, row_ptr, col_idx, s);
}

}  // namespace spmm
