// Pipelined block-sparse x dense SpMM for 16-bit X (FP16/BF16), block sizes
// 16 and 32, weights in FP16/BF16 or FP8-E4M3 with per-block FP32 scales.
//
// Y = (M o W) * X (PopSparse, Section 3), FP32 accumulation.
//
// A workgroup of 8 waves owns one panel of row groups (GR block rows each) and
// one n-tile of 16*NS columns, and walks the group's non-empty k-chunks (KC = 64
// k rows each). What a chunk needs is staged in LDS:
//   * the X rows of the chunk, row-major with a 16-byte XOR swizzle; each lane
//     fetches its MFMA B operand (4 consecutive k of one column) with the
//     transposing LDS read;
//   * the chunk's weight blocks (contiguous in the packed value buffer: the
//     plan buckets blocks by (group, chunk, row)), their block columns, the
//     per-row cell offsets and, for FP8, the block scales.
// Loading is spread over the waves: the four wave pairs take turns, each pair
// holding one whole chunk in registers from the moment it issues the loads
// until, four chunks later, it writes them into the LDS stage that is about to
// be multiplied. Four chunks are therefore in flight per workgroup while each
// wave only ever waits for its own single chunk. Buffer loads return zero out
// of range, which covers the k and n tails.
// Each wave keeps RW block rows x 16*NS columns of FP32 accumulators; two b=16
// blocks of a row share one 16x16x32 MFMA (their k ranges are concatenated).
// The epilogue rounds the accumulators into an LDS tile per wave and writes Y
// with 16-byte stores.
#pragma once

#include <type_traits>

#include "common.h"

namespace spmm {
namespace pipe {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
#define SPMM_LDS __attribute__((address_space(3)))

struct Fp8 {};  // weights stored as OCP E4M3FN codes

struct Params {
  KernelPlan kp;
  const void* W;          // packed values, entry order
  const float* scales;    // packed FP8 scales, entry order (or nullptr)
  const void* X;
  void* Y;
  int64_t ldx, ldy;
  int32_t n;
  int32_t num_units;
  uint32_t x_bytes;       // readable bytes of X (k * ldx * 2)
  uint32_t w_bytes;       // bytes of the packed values
  uint32_t nnz;           // entries
  const int32_t* status;  // skip when *status != 0 (dynamic), else nullptr
  const int32_t* ovf;     // skip when *ovf != 0 (a chunk too large for the stage), else nullptr
};

constexpr uint32_t kOOB = 0x80000000u;  // offset that lies outside every buffer used here

__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

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

// Four E4M3FN codes -> four values of XT (exact: 4 significant bits, range 2^-9..448).
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

template <typename XT, typename WT, typename YT, int B, int RW, int NS, int NWV>
struct Cfg {
  static constexpr bool kFp8 = __is_same(WT, Fp8);
  static constexpr int WAVES = 8, NT = 512, PL = 128;   // PL: lanes of one loading pair
  static constexpr int GR = WAVES * RW;
  static constexpr int NTILE = 16 * NS;
  static constexpr int KC = 64;                    // k rows per chunk
  static constexpr int CW = KC / B;                // block columns per chunk
  static constexpr int H = B / 16;                 // row tiles per block
  static constexpr int ROWB = NTILE * 2;           // bytes per X row in LDS
  static constexpr int CPR = ROWB / 16;            // 16-byte chunks per X row
  static constexpr int RP = 16 / CPR;              // X rows per 256 bytes
  static constexpr int X_BYTES = KC * ROWB;
  static constexpr int NXV = X_BYTES / (16 * PL);  // X vectors per loading lane
  static constexpr int WE = kFp8 ? 1 : 2;
  static constexpr int WB = B * B * WE;
  static constexpr int VPB = WB / 16;
  static constexpr int WCAP = NWV * PL / VPB;      // blocks staged per chunk
  static constexpr int W_OFF = X_BYTES;
  static constexpr int COL_OFF = W_OFF + NWV * PL * 16;
  static constexpr int CELL_OFF = COL_OFF + PL * 4;
  static constexpr int SC_OFF = CELL_OFF + PL * 4;
  static constexpr int STAGE = SC_OFF + (kFp8 ? PL * 4 : 0);
  static constexpr int NCH_MAX = 1024;
  // epilogue tile per wave: 16 rows x NTILE columns of YT, rows padded by 16 bytes
  static constexpr int ETROW = NTILE * (int)sizeof(YT) + 16;
  static constexpr int ETILE = 16 * ETROW;
  static constexpr int EPS = STAGE / ETILE;        // epilogue tiles per stage
  static_assert(NXV >= 1 && X_BYTES % (16 * PL) == 0, "X chunk must split evenly over a wave pair");
  static_assert(WCAP >= 1 && WCAP <= PL && (NWV * PL) % VPB == 0, "W stage");
  static_assert(GR + 1 <= PL, "cell offsets");
  static_assert(EPS >= 1 && EPS * 3 >= WAVES, "epilogue tiles must fit in three stages");
  static_assert(CPR == 8 || CPR == 16, "swizzle covers 128- or 256-byte rows");
};

// wait for every memory operation of this wave
__device__ __forceinline__ void wait_all() { __builtin_amdgcn_s_waitcnt(0); }
// Workgroup barrier that orders LDS traffic only: this wave's LDS operations
// are complete, loads into registers may still be in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __builtin_amdgcn_s_barrier();
}

// LDS: two stages for the chunk ring, a third used only by the epilogue, the
// chunk starts of the current group and the list of its non-empty chunks.
constexpr int kStageMax = 34304;
static __shared__ __attribute__((aligned(16))) uint8_t st0[kStageMax];
static __shared__ __attribute__((aligned(16))) uint8_t st1[kStageMax];
static __shared__ __attribute__((aligned(16))) uint8_t st2[kStageMax];
static __shared__ int32_t starts[1025];
static __shared__ int32_t nelist[1024];
static __shared__ int32_t scan_tmp[512];

__device__ __forceinline__ SPMM_LDS uint8_t* stage_ptr(int j) {
  return j == 0 ? (SPMM_LDS uint8_t*)st0 : j == 1 ? (SPMM_LDS uint8_t*)st1 : (SPMM_LDS uint8_t*)st2;
}

template <typename XT, typename WT, typename YT, int B, int RW, int NS, int NWV>
struct Kernel {
  using C = Cfg<XT, WT, YT, B, RW, NS, NWV>;

  // byte offset of (row, 16-byte chunk) in a swizzled X stage
  static __device__ __forceinline__ int xoff(int row, int chunk) {
    const int sw = 2 * ((row / C::RP) % (C::CPR / 2));
    return row * C::ROWB + ((chunk ^ sw) << 4);
  }

  // Transposing read: lane (g, t) receives B[k = kr + q][col = 16 s + t], q = 0..3.
  static __device__ __forceinline__ u32x2 btr(const SPMM_LDS uint8_t* st, int kr, int s, int t) {
    const int row = kr + (t >> 2);
    const int col = 16 * s + 4 * (t & 3);
    const int off = xoff(row, col >> 3) + ((col & 7) << 1);
    short4_t v = __builtin_amdgcn_ds_read_tr16_b64_v4i16((SPMM_LDS short4_t*)(st + off));
    return __builtin_bit_cast(u32x2, v);
  }

  // One chunk in the registers of a wave pair (lane lid in [0, 128)).
  struct Slot {
    u32x4 x[C::NXV];
    u32x4 w[NWV];
    int32_t col, cell, sc;
  };

  // Load chunk `ch` (entries [e0, e0 + cnt), cnt <= WCAP) into the pair's
  // registers. Lanes with nothing to fetch read out of range and get zeros.
  static __device__ __forceinline__ void load(Slot& sl, const Params& p, int lid, int32_t grp, int32_t ch,
                                              int32_t e0, int32_t cnt, int32_t n0) {
    const KernelPlan& kp = p.kp;
    __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)p.X, (short)0, (int)p.x_bytes, 0x00020000);
    __amdgpu_buffer_rsrc_t wr = __builtin_amdgcn_make_buffer_rsrc((void*)p.W, (short)0, (int)p.w_bytes, 0x00020000);
#pragma unroll
    for (int i = 0; i < C::NXV; ++i) {
      const int v = i * C::PL + lid;
      const int row = v / C::CPR, pos = v % C::CPR;
      const int sw = 2 * ((row / C::RP) % (C::CPR / 2));
      const int lc = pos ^ sw;
      const int64_t krow = (int64_t)ch * C::KC + row;
      const uint32_t off = krow < kp.k ? (uint32_t)((krow * p.ldx + n0 + lc * 8) * 2) : kOOB;
      sl.x[i] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(xr, off, 0, 0));
    }
#pragma unroll
    for (int i = 0; i < NWV; ++i) {
      const int v = i * C::PL + lid;
      const uint32_t off = v < cnt * C::VPB ? (uint32_t)((int64_t)e0 * C::WB + v * 16) : kOOB;
      sl.w[i] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(wr, off, 0, 0));
    }
    __amdgpu_buffer_rsrc_t cr = __builtin_amdgcn_make_buffer_rsrc((void*)kp.ent_col, (short)0, (int)(p.nnz * 4u), 0x00020000);
    sl.col = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(cr, lid < cnt ? (uint32_t)(e0 + lid) * 4u : kOOB, 0, 0);
    const uint32_t ncell_bytes = (uint32_t)(((int64_t)kp.num_groups * kp.num_chunks * kp.group_rows + 1) * 4);
    __amdgpu_buffer_rsrc_t pr = __builtin_amdgcn_make_buffer_rsrc((void*)kp.cell_ptr, (short)0, (int)ncell_bytes, 0x00020000);
    const uint32_t coff = lid <= C::GR ? (uint32_t)((((int64_t)grp * kp.num_chunks + ch) * C::GR + lid) * 4) : kOOB;
    sl.cell = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(pr, coff, 0, 0);
    if constexpr (C::kFp8) {
      __amdgpu_buffer_rsrc_t sr = __builtin_amdgcn_make_buffer_rsrc((void*)p.scales, (short)0, (int)(p.nnz * 4u), 0x00020000);
      sl.sc = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(sr, lid < cnt ? (uint32_t)(e0 + lid) * 4u : kOOB, 0, 0);
    } else {
      sl.sc = 0;
    }
  }

  // Write the pair's chunk into an LDS stage (X keeps the swizzled layout).
  static __device__ __forceinline__ void store(SPMM_LDS uint8_t* st, const Slot& sl, int lid) {
#pragma unroll
    for (int i = 0; i < C::NXV; ++i) *(SPMM_LDS u32x4*)(st + (i * C::PL + lid) * 16) = sl.x[i];
#pragma unroll
    for (int i = 0; i < NWV; ++i) *(SPMM_LDS u32x4*)(st + C::W_OFF + (i * C::PL + lid) * 16) = sl.w[i];
    ((SPMM_LDS int32_t*)(st + C::COL_OFF))[lid] = sl.col;
    ((SPMM_LDS int32_t*)(st + C::CELL_OFF))[lid] = sl.cell;
    if constexpr (C::kFp8) ((SPMM_LDS int32_t*)(st + C::SC_OFF))[lid] = sl.sc;
  }

  template <typename V>
  static __device__ __forceinline__ V wfrag(const SPMM_LDS uint8_t* st, int32_t q, int off) {
    return *(const SPMM_LDS V*)(st + C::W_OFF + q * C::WB + off);
  }

  // Multiply the chunk staged in `st` into the accumulators of this wave's rows.
  static __device__ __forceinline__ void compute(const SPMM_LDS uint8_t* st, int32_t ch, int32_t e0,
                                                 float4_t (&acc)[RW][B / 16][NS]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, t = lane & 15;
    const int32_t cbase = ch * C::CW;
    const SPMM_LDS int32_t* cell = (const SPMM_LDS int32_t*)(st + C::CELL_OFF);
    const SPMM_LDS int32_t* cols = (const SPMM_LDS int32_t*)(st + C::COL_OFF);
    int32_t cb[RW + 1];
#pragma unroll
    for (int r = 0; r <= RW; ++r) cb[r] = uniform(cell[wave * RW + r]) - e0;
    // the wave's block columns (and scales), one lane per entry
    const int32_t qlo = cb[0];
    const int32_t colv = cols[min(qlo + lane, C::PL - 1)] - cbase;
    float scv = 0.f;
    if constexpr (C::kFp8) scv = ((const SPMM_LDS float*)(st + C::SC_OFF))[min(qlo + lane, C::PL - 1)];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int32_t q0 = cb[r], q1 = cb[r + 1];
      if constexpr (!C::kFp8 && B == 16) {
        for (int32_t q = q0; q < q1; q += 2) {
          const bool two = q + 1 < q1;
          const int32_t c1 = __builtin_amdgcn_readlane(colv, q - qlo);
          const int32_t c2 = two ? __builtin_amdgcn_readlane(colv, q + 1 - qlo) : c1;
          const u32x2 a1 = wfrag<u32x2>(st, q, (t * 16 + g * 4) * 2);
          const u32x2 a2 = two ? wfrag<u32x2>(st, q + 1, (t * 16 + g * 4) * 2) : u32x2{0u, 0u};
          const u32x4 a = {a1.x, a1.y, a2.x, a2.y};
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const u32x2 b1 = btr(st, c1 * 16 + 4 * g, s, t);
            const u32x2 b2 = two ? btr(st, c2 * 16 + 4 * g, s, t) : u32x2{0u, 0u};
            acc[r][0][s] = Mma<XT>::k32(a, u32x4{b1.x, b1.y, b2.x, b2.y}, acc[r][0][s]);
          }
        }
      } else if constexpr (!C::kFp8) {  // B == 32, 16-bit weights
        for (int32_t q = q0; q < q1; ++q) {
          const int32_t c = __builtin_amdgcn_readlane(colv, q - qlo);
#pragma unroll
          for (int h = 0; h < C::H; ++h) {
            const u32x4 a = wfrag<u32x4>(st, q, ((h * 16 + t) * B + g * 8) * 2);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
              const u32x2 b1 = btr(st, c * B + 8 * g, s, t);
              const u32x2 b2 = btr(st, c * B + 8 * g + 4, s, t);
              acc[r][h][s] = Mma<XT>::k32(a, u32x4{b1.x, b1.y, b2.x, b2.y}, acc[r][h][s]);
            }
          }
        }
      } else {  // FP8 weights with a per-block scale
        for (int32_t q = q0; q < q1; ++q) {
          const int32_t c = __builtin_amdgcn_readlane(colv, q - qlo);
          const float sc = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int32_t, scv), q - qlo));
#pragma unroll
          for (int h = 0; h < C::H; ++h) {
            if constexpr (B == 16) {
              const u32x2 a = fp8x4<XT>(wfrag<uint32_t>(st, q, t * 16 + g * 4));
#pragma unroll
              for (int s = 0; s < NS; ++s) {
                const u32x2 bx = btr(st, c * 16 + 4 * g, s, t);
                const float4_t part = Mma<XT>::k16(a, bx, float4_t{0.f, 0.f, 0.f, 0.f});
                acc[r][h][s] += sc * part;
              }
            } else {
              const u32x2 codes = wfrag<u32x2>(st, q, (h * 16 + t) * B + g * 8);
              const u32x2 lo = fp8x4<XT>(codes.x), hi = fp8x4<XT>(codes.y);
              const u32x4 a = {lo.x, lo.y, hi.x, hi.y};
#pragma unroll
              for (int s = 0; s < NS; ++s) {
                const u32x2 b1 = btr(st, c * B + 8 * g, s, t);
                const u32x2 b2 = btr(st, c * B + 8 * g + 4, s, t);
                const float4_t part = Mma<XT>::k32(a, u32x4{b1.x, b1.y, b2.x, b2.y}, float4_t{0.f, 0.f, 0.f, 0.f});
                acc[r][h][s] += sc * part;
              }
            }
          }
        }
      }
    }
  }

  // Round a wave's accumulators into its LDS tile (16 rows at a time) and write
  // Y with 16-byte stores; rows >= m and columns >= n are not written.
  static __device__ __forceinline__ void epilogue(SPMM_LDS uint8_t* tile, const Params& p, int32_t grp, int32_t n0,
                                                  const float4_t (&acc)[RW][B / 16][NS]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, t = lane & 15;
    constexpr int YS = (int)sizeof(YT);
    constexpr int EPV = 16 / YS;                       // elements per 16-byte store
    constexpr int VPR = C::NTILE / EPV;                // 16-byte vectors per row
    YT* __restrict__ Y = (YT*)p.Y;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
#pragma unroll
      for (int h = 0; h < C::H; ++h) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float v = acc[r][h][s][i];
            *(SPMM_LDS YT*)(tile + (4 * g + i) * C::ETROW + (16 * s + t) * YS) = to_out<YT>(v);
          }
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): the tile is complete before it is read back
        const int64_t row0 = ((int64_t)grp * C::GR + wave * RW + r) * B + h * 16;
#pragma unroll
        for (int it = 0; it < (16 * VPR) / 64; ++it) {
          const int idx = it * 64 + lane;
          const int rr = idx / VPR, cv = idx % VPR;
          const int64_t row = row0 + rr;
          const int32_t col = n0 + cv * EPV;
          const u32x4 v = *(const SPMM_LDS u32x4*)(tile + rr * C::ETROW + cv * 16);
          if (row < p.kp.m) {
            YT* dst = Y + row * p.ldy + col;
            if (col + EPV <= p.n) {
              *(u32x4*)dst = v;
            } else if (col < p.n) {
              YT tmp[EPV];
              __builtin_memcpy(tmp, &v, 16);
#pragma unroll
              for (int e = 0; e < EPV; ++e)
                if (col + e < p.n) dst[e] = tmp[e];
            }
          }
        }
        __builtin_amdgcn_s_waitcnt(0xC07F);  // reads done before the next tile overwrites it
      }
    }
  }
};

template <typename XT, typename WT, typename YT, int B, int RW, int NS, int NWV>
__global__ __launch_bounds__(512) void k_spmm_pipe(Params p) {
  using K = Kernel<XT, WT, YT, B, RW, NS, NWV>;
  using C = typename K::C;
  static_assert(C::STAGE <= kStageMax, "stage larger than the LDS ring slots");
  if ((p.status && *p.status) || (p.ovf && *p.ovf)) return;

  const int tid = threadIdx.x, wave = tid >> 6;
  const int pair = wave >> 1, lid = tid & 127;
  const KernelPlan& kp = p.kp;
  const int32_t NCH = kp.num_chunks;
  const int32_t unit = xcd_unit(blockIdx.x, p.num_units);
  const int32_t panel = unit % kp.num_panels;
  const int32_t n0 = (unit / kp.num_panels) * C::NTILE;

  float4_t acc[RW][B / 16][NS];
  typename K::Slot sl;
  const int32_t g_lo = kp.panel_ptr[panel], g_hi = kp.panel_ptr[panel + 1];
  for (int32_t grp = g_lo; grp < g_hi; ++grp) {
    // chunk starts of this group, then the compacted list of its non-empty chunks
    for (int32_t c = tid; c <= NCH; c += C::NT) starts[c] = kp.cell_ptr[((int64_t)grp * NCH + c) * C::GR];
    wait_all();
    __syncthreads();
    const int32_t c0 = 2 * tid, c1 = 2 * tid + 1;
    const int f0 = c0 < NCH && starts[c0 + 1] > starts[c0];
    const int f1 = c1 < NCH && starts[c1 + 1] > starts[c1];
    scan_tmp[tid] = f0 + f1;
    __syncthreads();
    for (int off = 1; off < C::NT; off <<= 1) {
      const int add = tid >= off ? scan_tmp[tid - off] : 0;
      __syncthreads();
      scan_tmp[tid] += add;
      __syncthreads();
    }
    const int32_t incl = scan_tmp[tid];
    const int32_t N = uniform(scan_tmp[C::NT - 1]);
    if (f0) nelist[incl - f0 - f1] = c0;
    if (f1) nelist[incl - f1] = c1;
    __syncthreads();

#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int h = 0; h < B / 16; ++h)
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[r][h][s] = float4_t{0.f, 0.f, 0.f, 0.f};

    // sequence index i -> chunk nelist[i]; pair (i mod 4) loads it
    auto load_seq = [&](int32_t i) {
      if (i < N) {
        const int32_t ch = nelist[i];
        K::load(sl, p, lid, grp, ch, starts[ch], starts[ch + 1] - starts[ch], n0);
      }
    };
    load_seq(pair);
    if (pair == 0) {
      if (N > 0) {
        wait_all();
        K::store(stage_ptr(0), sl, lid);
      }
      load_seq(4);
    }
    lds_barrier();
    for (int32_t i = 0; i < N; ++i) {
      if (pair == ((i + 1) & 3)) {
        if (i + 1 < N) {
          wait_all();
          K::store(stage_ptr((i + 1) & 1), sl, lid);
        }
        load_seq(i + 5);
      }
      const int32_t ch = nelist[i];
      K::compute(stage_ptr(i & 1), ch, starts[ch], acc);
      lds_barrier();
    }
    wait_all();
    __syncthreads();
    // epilogue through LDS (the stages are idle now)
    SPMM_LDS uint8_t* tile = stage_ptr(wave / C::EPS) + (wave % C::EPS) * C::ETILE;
    K::epilogue(tile, p, grp, n0, acc);
    wait_all();
    __syncthreads();
  }
}

template <typename XT, typename WT, typename YT, int B, int RW, int NS, int NWV>
spmm_status_t launch_pipe(const RunArgs& a, hipStream_t stream) {
  using C = Cfg<XT, WT, YT, B, RW, NS, NWV>;
  Params p;
  p.kp = a.plan;
  p.W = a.W;
  p.scales = a.scales;
  p.X = a.X;
  p.Y = a.Y;
  p.ldx = a.ldx;
  p.ldy = a.ldy;
  p.n = a.n;
  p.status = a.status;
  p.ovf = a.ovf_mode == 1 ? a.ovf : nullptr;
  p.x_bytes = (uint32_t)((int64_t)a.plan.k * a.ldx * 2);
  p.nnz = (uint32_t)a.nnz;
  p.w_bytes = (uint32_t)(a.nnz * (int64_t)C::WB);
  const int64_t units = ceil_div(a.n, C::NTILE) * (int64_t)a.plan.num_panels;
  if (units == 0) return SPMM_OK;
  p.num_units = (int32_t)units;
  hipLaunchKernelGGL((k_spmm_pipe<XT, WT, YT, B, RW, NS, NWV>), dim3((unsigned)units), dim3(512), 0, stream, p);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

}  // namespace pipe
}  // namespace spmm
