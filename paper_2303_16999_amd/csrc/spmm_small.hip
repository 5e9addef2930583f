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
};

constexpr uint32_t kOOB = 0x80000000u;
constexpr int kRowsPerWg = 4;  // one block row per wave

__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int32_t xcd_unit(int32_t w, int32_t U) {
  const int32_t q = U >> 3, r = U & 7;
  const int32_t x = w & 7, local = w >> 3;
  return x * q + min(x, r) + local;
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
  const int32_t rg = unit % rgroups;
  const int32_t n0 = (unit / rgroups) * (64 * V);
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
  const int64_t xb = (int64_t)a.plan.k * a.ldx * (int64_t)sizeof(XT);
  if (xb >= (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "X larger than 2 GiB is not supported");
  p.x_bytes = (uint32_t)xb;
  const int64_t units = ceil_div(a.plan.mb, kRowsPerWg) * ceil_div(a.n, 64 * V);
  if (units == 0) return SPMM_OK;
  if (units > (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "too many work units");
  p.num_units = (int32_t)units;
  hipLaunchKernelGGL((k_spmm_small<XT, WT, YT, B, V>), dim3((unsigned)units), dim3(256), 0, s, p);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

// columns per lane: the requested variant (4 or 8), else 8 (16-byte loads of
// 16-bit X) unless n is small enough that a 256-column tile already covers it
template <typename XT, typename WT, typename YT, int B>
spmm_status_t small_v(const RunArgs& a, const int32_t* rp, const int32_t* ci, hipStream_t s) {
  if constexpr (sizeof(XT) == 4) return launch_small<XT, WT, YT, B, 4>(a, rp, ci, s);
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
