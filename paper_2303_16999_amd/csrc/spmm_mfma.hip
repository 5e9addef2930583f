// Block-sparse x dense SpMM on MFMA for block sizes 16 and 32 (gfx950).
//
// Computes Y = (M o W) * X (PopSparse, Section 3) with FP32 accumulation.
// A workgroup owns one panel of row groups and one n-tile of 16*NS columns.
// For each group it walks k in chunks of CW block columns; a chunk stages in
// LDS:
//   * the X rows of the chunk, transposed so that every column's k values are
//     contiguous (one 8- or 16-byte LDS read gives a lane its MFMA operand);
//   * the group's nonzero blocks that fall in the chunk (contiguous in the
//     packed value buffer because the plan buckets blocks by (group, chunk,
//     row)), their block columns, and the per-row cell offsets.
// Each wave keeps RW block rows x 16*NS columns of FP32 accumulators in
// registers and walks its rows' blocks; every block contributes b/16 row tiles
// x NS MFMA column tiles. Two b=16 blocks of one row are fused into one
// 16x16x32 MFMA (their k ranges are concatenated), which runs at twice the
// rate of the 16x16x16 form on gfx950. The next chunk's global loads are in
// flight while the current chunk computes (register double buffering into a
// second LDS stage).
//
// Lane mapping (MFMA 16x16xK, 64 lanes, g = lane / 16, j = lane % 16):
//   A operand row j   = block row j of the current row tile;
//   B operand column j of column tile s = physical column j*NS + s of the
//     n-tile, so a lane's accumulators over s are NS consecutive columns of Y
//     and the epilogue writes 2*NS (or 4*NS) contiguous bytes per row;
//   k values held by lane group g for one block = block columns
//     [g*b/4, (g+1)*b/4) (any assignment works as long as A and B agree).
#include "common.h"

namespace spmm {
namespace {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct Fp8Tag {};  // W stored as OCP E4M3FN codes

struct Params {
  KernelPlan kp;
  const void* W;
  const float* scales;
  const void* X;
  void* Y;
  int64_t ldx, ldy;
  int32_t n;
  int32_t ntiles;
  int32_t num_units;
  const int32_t* status;
  const int32_t* ovf_only;  // run only when *ovf_only != 0 (fallback for oversized chunks), else nullptr
};

// Global load for the rare path of blocks that did not fit the LDS stage. A
// buffer load cannot be folded with the LDS load of the common path into one
// generic-address load (which the backend miscompiles). Offsets stay below 2 GiB.
template <typename V>
__device__ __forceinline__ V load_slow(const V* ptr) {
  __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void*)ptr, (short)0, 0x7FFFFFFF, 0x00020000);
  if constexpr (sizeof(V) == 4) return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, 0, 0, 0));
  else if constexpr (sizeof(V) == 8) return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  else return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
}

__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// XCD-aware unit order: workgroup w runs on XCD w % 8. Consecutive logical
// units (which share an n-tile, so the same X columns) are given to the same
// XCD and therefore share its L2.
__device__ __forceinline__ int32_t xcd_unit(int32_t w, int32_t U) {
  const int32_t q = U >> 3, r = U & 7;
  const int32_t x = w & 7, local = w >> 3;
  return x * q + min(x, r) + local;
}

// ---------------------------------------------------------------- MFMA wrappers
template <typename XT> struct Mfma;
template <> struct Mfma<_Float16> {
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
template <> struct Mfma<__bf16> {
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

// Four E4M3FN codes (one dword) -> four 16-bit values of XT, exactly.
template <typename XT>
__device__ __forceinline__ u32x2 fp8x4_to(uint32_t codes) {
  auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)codes, false);
  auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)codes, true);
  u32x2 r;
  r.x = Mfma<XT>::pack2(lo[0], lo[1]);
  r.y = Mfma<XT>::pack2(hi[0], hi[1]);
  return r;
}

template <typename YT> __device__ __forceinline__ YT cvt_out(float v);
template <> __device__ __forceinline__ float cvt_out<float>(float v) { return v; }
template <> __device__ __forceinline__ _Float16 cvt_out<_Float16>(float v) { return (_Float16)v; }
template <> __device__ __forceinline__ __bf16 cvt_out<__bf16>(float v) { return (__bf16)v; }

// ---------------------------------------------------------------- the kernel
template <typename XT, typename WT, typename YT, int B, int WAVES, int RW, int NS, int CW, int WCAP, bool GATHER>
struct Cfg {
  static constexpr bool kFp8 = __is_same(WT, Fp8Tag);
  static constexpr bool kF32 = __is_same(XT, float);
  static constexpr int NT = WAVES * 64;
  static constexpr int GR = WAVES * RW;          // block rows per group
  static constexpr int NTILE = 16 * NS;          // columns per workgroup
  static constexpr int KC = CW * B;              // k rows per chunk
  static constexpr int XE = sizeof(XT);
  static constexpr int VEC = 16 / XE;            // X elements per 16-byte vector
  static constexpr int KCP = KC + VEC;           // padded Xt row (elements)
  static constexpr int H = B / 16;               // row tiles per block
  static constexpr int KL = B / 4;               // k values per lane per block
  static constexpr int WE = kFp8 ? 1 : XE;       // bytes per stored weight
  static constexpr int WB = B * B * WE;          // bytes per block
  static constexpr int VPB = WB / 16;            // 16-byte vectors per block
  static constexpr int NWV = (WCAP * VPB + NT - 1) / NT;   // W vectors per thread
  static constexpr int XTASKS = (KC / 8) * (NTILE / VEC);  // 8 rows x VEC columns each
  static constexpr int NXT = (XTASKS + NT - 1) / NT;
  static constexpr bool kPair = !kF32 && !kFp8 && B == 16;
  // LDS stage layout (bytes)
  static constexpr int XT_BYTES = NTILE * KCP * XE;
  static constexpr int W_OFF = XT_BYTES;
  static constexpr int COL_OFF = W_OFF + WCAP * WB;
  static constexpr int CELL_OFF = COL_OFF + WCAP * 4;
  static constexpr int SC_OFF = CELL_OFF + (GR + 1) * 4;
  static constexpr int STAGE = ((SC_OFF + (kFp8 ? WCAP * 4 : 0)) + 15) / 16 * 16;
  static constexpr int LDS = 2 * STAGE;
  static_assert(KC % 8 == 0, "chunk must hold a multiple of 8 k rows");
  static_assert(NTILE % VEC == 0, "tile width");
  static_assert(LDS <= 160 * 1024, "LDS budget");
  static_assert(WB % 16 == 0, "block bytes");
  static_assert(NT >= WCAP + GR + 1, "metadata staging needs one thread per entry");
  static_assert(NS % 2 == 0, "column tile");
};

template <typename XT, typename WT, typename YT, int B, int WAVES, int RW, int NS, int CW, int WCAP, bool GATHER>
__global__ __launch_bounds__(WAVES * 64) void k_spmm_mfma(Params p) {
  using C = Cfg<XT, WT, YT, B, WAVES, RW, NS, CW, WCAP, GATHER>;
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  if (p.status && *p.status) return;
  if (p.ovf_only && !*p.ovf_only) return;

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, j = lane & 15;
  const KernelPlan& kp = p.kp;
  const int32_t NCH = kp.num_chunks;
  const int32_t unit = xcd_unit(blockIdx.x, p.num_units);
  const int32_t panel = unit % kp.num_panels;
  const int32_t tile = unit / kp.num_panels;
  const int32_t n0 = tile * C::NTILE;
  const XT* __restrict__ X = (const XT*)p.X;
  const uint8_t* __restrict__ Wb = (const uint8_t*)p.W;
  const int32_t krem = kp.k - (kp.k / B) * B;

  // prefetch registers
  u32x4 xr[C::NXT][8];
  u32x4 wr[C::NWV];
  int32_t meta_col = 0, meta_cell = 0;
  float meta_sc = 0.f;

  // ---- global -> registers for chunk (grp, ch)
  auto load_stage = [&](int32_t grp, int32_t ch, int32_t e0, int32_t cnt) {
    // X: task t covers k rows ch*KC + kg*8 + [0,8) and columns n0 + cg*VEC + [0,VEC)
#pragma unroll
    for (int s = 0; s < C::NXT; ++s) {
      const int t = tid + s * C::NT;
      const int kg = t / (C::NTILE / C::VEC), cg = t % (C::NTILE / C::VEC);
      const int32_t col = n0 + cg * C::VEC;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int32_t row = ch * C::KC + kg * 8 + i;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (t < C::XTASKS && row < kp.k) {
          const XT* src = X + (int64_t)row * p.ldx + col;
          if (col + C::VEC <= p.n) {
            v = *(const u32x4*)src;
          } else if (col < p.n) {
            XT tmp[C::VEC];
#pragma unroll
            for (int q = 0; q < C::VEC; ++q) tmp[q] = (col + q < p.n) ? src[q] : XT(0);
            v = __builtin_bit_cast(u32x4, tmp);
          }
        }
        xr[s][i] = v;
      }
    }
    // W: the chunk's staged blocks are entries [e0, e0 + min(cnt, WCAP))
    const int32_t staged = min(cnt, WCAP);
#pragma unroll
    for (int s = 0; s < C::NWV; ++s) {
      const int v = tid + s * C::NT;
      u32x4 val = {0u, 0u, 0u, 0u};
      if (v < staged * C::VPB) {
        const int32_t q = v / C::VPB, vi = v % C::VPB;
        const int32_t e = e0 + q;
        const int64_t src_blk = GATHER ? (int64_t)kp.ent_src[e] : (int64_t)e;
        val = *(const u32x4*)(Wb + src_blk * C::WB + vi * 16);
        if (GATHER && krem && kp.ent_col[e] == kp.kb - 1) {
          // zero the part of an edge block that lies beyond column k
          constexpr int EPV = 16 / C::WE;
          uint8_t bytes[16];
          __builtin_memcpy(bytes, &val, 16);
#pragma unroll
          for (int q2 = 0; q2 < EPV; ++q2) {
            const int colb = (vi * EPV + q2) % B;
            if (colb >= krem)
#pragma unroll
              for (int z = 0; z < C::WE; ++z) bytes[q2 * C::WE + z] = 0;
          }
          __builtin_memcpy(&val, bytes, 16);
        }
      }
      wr[s] = val;
    }
    // metadata
    if (tid < WCAP) {
      meta_col = tid < staged ? kp.ent_col[e0 + tid] : 0;
      if constexpr (C::kFp8) {
        const int32_t e = e0 + tid;
        meta_sc = tid < staged ? p.scales[GATHER ? kp.ent_src[e] : e] : 0.f;
      }
    } else if (tid < WCAP + C::GR + 1) {
      meta_cell = kp.cell_ptr[((int64_t)grp * NCH + ch) * C::GR + (tid - WCAP)] - e0;
    }
  };

  // ---- registers -> LDS stage
  auto store_stage = [&](int buf) {
    uint8_t* st = lds + buf * C::STAGE;
    XT* xt = (XT*)st;
#pragma unroll
    for (int s = 0; s < C::NXT; ++s) {
      const int t = tid + s * C::NT;
      if (t < C::XTASKS) {
        const int kg = t / (C::NTILE / C::VEC), cg = t % (C::NTILE / C::VEC);
        if constexpr (C::kF32) {
          // 8 rows x 4 floats -> 4 columns x 8 floats
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int pc = cg * 4 + q;
            const int mcol = (pc % NS) * 16 + pc / NS;
            u32x4 lo = {xr[s][0][q], xr[s][1][q], xr[s][2][q], xr[s][3][q]};
            u32x4 hi = {xr[s][4][q], xr[s][5][q], xr[s][6][q], xr[s][7][q]};
            u32x4* dst = (u32x4*)(xt + mcol * C::KCP + kg * 8);
            dst[0] = lo;
            dst[1] = hi;
          }
        } else {
          // 8 rows x 8 halves -> 8 columns x 8 halves (16-bit transpose with v_perm)
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const int pc = cg * 8 + q;
            const int mcol = (pc % NS) * 16 + pc / NS;
            const uint32_t sel = (q & 1) ? 0x07060302u : 0x05040100u;
            u32x4 o;
            o.x = __builtin_amdgcn_perm(xr[s][1][q >> 1], xr[s][0][q >> 1], sel);
            o.y = __builtin_amdgcn_perm(xr[s][3][q >> 1], xr[s][2][q >> 1], sel);
            o.z = __builtin_amdgcn_perm(xr[s][5][q >> 1], xr[s][4][q >> 1], sel);
            o.w = __builtin_amdgcn_perm(xr[s][7][q >> 1], xr[s][6][q >> 1], sel);
            *(u32x4*)(xt + mcol * C::KCP + kg * 8) = o;
          }
        }
      }
    }
    u32x4* wst = (u32x4*)(st + C::W_OFF);
#pragma unroll
    for (int s = 0; s < C::NWV; ++s) {
      const int v = tid + s * C::NT;
      if (v < WCAP * C::VPB) wst[v] = wr[s];
    }
    if (tid < WCAP) {
      ((int32_t*)(st + C::COL_OFF))[tid] = meta_col;
      if constexpr (C::kFp8) ((float*)(st + C::SC_OFF))[tid] = meta_sc;
    } else if (tid < WCAP + C::GR + 1) {
      ((int32_t*)(st + C::CELL_OFF))[tid - WCAP] = meta_cell;
    }
  };

  // ---- fragment loaders (entry q relative to the chunk's first entry e0)
  // W fragment of staged entry q at byte offset off inside the block: from the
  // LDS stage when q was staged, else straight from global memory.
  auto w_load = [&](const uint8_t* st, int32_t e0, int32_t q, int off, auto tag) {
    using V = decltype(tag);
    if (q < WCAP) return *(const V*)(st + C::W_OFF + q * C::WB + off);
    const int32_t e = e0 + q;
    return load_slow((const V*)(Wb + (int64_t)(GATHER ? kp.ent_src[e] : e) * C::WB + off));
  };
  auto col_of = [&](const uint8_t* st, int32_t e0, int32_t q) -> int32_t {
    return uniform(q < WCAP ? ((const int32_t*)(st + C::COL_OFF))[q] : kp.ent_col[e0 + q]);
  };

  float4_t acc[RW][C::H][NS];

  const int32_t g_lo = kp.panel_ptr[panel], g_hi = kp.panel_ptr[panel + 1];
  for (int32_t grp = g_lo; grp < g_hi; ++grp) {
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int h = 0; h < C::H; ++h)
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[r][h][s] = float4_t{0.f, 0.f, 0.f, 0.f};

    const int64_t gbase = (int64_t)grp * NCH * C::GR;
    auto chunk_start = [&](int32_t ch) -> int32_t { return kp.cell_ptr[gbase + (int64_t)ch * C::GR]; };
    // first non-empty chunk at or after ch
    auto next_chunk = [&](int32_t ch, int32_t& e0, int32_t& cnt) -> int32_t {
      int32_t a = ch < NCH ? chunk_start(ch) : 0;
      while (ch < NCH) {
        const int32_t b2 = chunk_start(ch + 1);
        if (b2 > a) { e0 = a; cnt = b2 - a; return ch; }
        a = b2;
        ++ch;
      }
      return NCH;
    };

    int32_t e0 = 0, cnt = 0;
    int32_t ch = next_chunk(0, e0, cnt);
    if (ch < NCH) {
      load_stage(grp, ch, e0, cnt);
      store_stage(0);
    }
    __syncthreads();
    int buf = 0;
    while (ch < NCH) {
      int32_t ne0 = 0, ncnt = 0;
      const int32_t nch = next_chunk(ch + 1, ne0, ncnt);
      if (nch < NCH) load_stage(grp, nch, ne0, ncnt);

      // ---- compute on stage `buf`
      const uint8_t* st = lds + buf * C::STAGE;
      const XT* xt = (const XT*)st;
      const int32_t* cellofs = (const int32_t*)(st + C::CELL_OFF);
      const int32_t cbase = ch * CW;
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        const int lr = wave * RW + r;
        const int32_t q0 = uniform(cellofs[lr]), q1 = uniform(cellofs[lr + 1]);
        if constexpr (C::kPair) {
          for (int32_t q = q0; q < q1; q += 2) {
            const bool two = q + 1 < q1;
            const int32_t c1 = col_of(st, e0, q) - cbase;
            const int32_t c2 = two ? col_of(st, e0, q + 1) - cbase : c1;
            u32x2 a1 = w_load(st, e0, q, (j * 16 + g * 4) * 2, u32x2{});
            u32x2 a2 = {0u, 0u};
            if (two) a2 = w_load(st, e0, q + 1, (j * 16 + g * 4) * 2, u32x2{});
            const u32x4 a = {a1.x, a1.y, a2.x, a2.y};
#pragma unroll
            for (int s = 0; s < NS; ++s) {
              const XT* xrow = xt + (s * 16 + j) * C::KCP + g * 4;
              u32x2 b1 = *(const u32x2*)(xrow + c1 * 16);
              u32x2 b2 = {0u, 0u};
              if (two) b2 = *(const u32x2*)(xrow + c2 * 16);
              const u32x4 bb = {b1.x, b1.y, b2.x, b2.y};
              acc[r][0][s] = Mfma<XT>::k32(a, bb, acc[r][0][s]);
            }
          }
        } else {
          for (int32_t q = q0; q < q1; ++q) {
            const int32_t c = col_of(st, e0, q) - cbase;
            float sc = 1.f;
            if constexpr (C::kFp8) {
              if (q < WCAP) sc = ((const float*)(st + C::SC_OFF))[q];
              else sc = load_slow(p.scales + (GATHER ? kp.ent_src[e0 + q] : e0 + q));
            }
#pragma unroll
            for (int h = 0; h < C::H; ++h) {
              const int wrow = h * 16 + j;
              if constexpr (C::kF32) {
                // KL = B/4 floats per lane: B/4 MFMAs of K = 4
#pragma unroll
                for (int v4 = 0; v4 < C::KL / 4; ++v4) {
                  const float4_t a = w_load(st, e0, q, (wrow * B + g * C::KL + v4 * 4) * 4, float4_t{});
#pragma unroll
                  for (int s = 0; s < NS; ++s) {
                    const float4_t bx = *(const float4_t*)(xt + (s * 16 + j) * C::KCP + c * B + g * C::KL + v4 * 4);
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                      acc[r][h][s] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], bx[t], acc[r][h][s], 0, 0, 0);
                  }
                }
              } else if constexpr (C::kFp8) {
                if constexpr (B == 16) {
                  const uint32_t codes = w_load(st, e0, q, wrow * B + g * 4, uint32_t{});
                  const u32x2 a = fp8x4_to<XT>(codes);
#pragma unroll
                  for (int s = 0; s < NS; ++s) {
                    const u32x2 bx = *(const u32x2*)(xt + (s * 16 + j) * C::KCP + c * B + g * 4);
                    const float4_t part = Mfma<XT>::k16(a, bx, float4_t{0.f, 0.f, 0.f, 0.f});
                    acc[r][h][s] += sc * part;
                  }
                } else {
                  const u32x2 codes = w_load(st, e0, q, wrow * B + g * 8, u32x2{});
                  const u32x2 lo = fp8x4_to<XT>(codes.x), hi = fp8x4_to<XT>(codes.y);
                  const u32x4 a = {lo.x, lo.y, hi.x, hi.y};
#pragma unroll
                  for (int s = 0; s < NS; ++s) {
                    const u32x4 bx = *(const u32x4*)(xt + (s * 16 + j) * C::KCP + c * B + g * 8);
                    const float4_t part = Mfma<XT>::k32(a, bx, float4_t{0.f, 0.f, 0.f, 0.f});
                    acc[r][h][s] += sc * part;
                  }
                }
              } else {
                // 16-bit, B = 32: KL = 8 -> one K = 32 MFMA per tile
                const u32x4 a = w_load(st, e0, q, (wrow * B + g * 8) * 2, u32x4{});
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                  const u32x4 bx = *(const u32x4*)(xt + (s * 16 + j) * C::KCP + c * B + g * 8);
                  acc[r][h][s] = Mfma<XT>::k32(a, bx, acc[r][h][s]);
                }
              }
            }
          }
        }
      }

      if (nch < NCH) store_stage(buf ^ 1);
      __syncthreads();
      ch = nch;
      e0 = ne0;
      cnt = ncnt;
      buf ^= 1;
    }

    // ---- epilogue: rows (grp*GR + wave*RW + r)*B + 16h + 4g + i, columns n0 + j*NS + s
    YT* __restrict__ Y = (YT*)p.Y;
    const int32_t col0 = n0 + j * NS;
#pragma unroll
    for (int r = 0; r < RW; ++r) {
#pragma unroll
      for (int h = 0; h < C::H; ++h) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t row = ((int64_t)grp * C::GR + wave * RW + r) * B + h * 16 + g * 4 + i;
          if (row >= kp.m) continue;
          YT* dst = Y + row * p.ldy + col0;
          if (col0 + NS <= p.n) {
            constexpr int WORDS = NS * (int)sizeof(YT) / 4;
            uint32_t words[WORDS];
#pragma unroll
            for (int w2 = 0; w2 < WORDS; ++w2) {
              if constexpr (sizeof(YT) == 4) {
                const float v = acc[r][h][w2][i];  // bit_cast of a vector element lvalue would read element 0
                words[w2] = __builtin_bit_cast(uint32_t, v);
              } else {
                const YT lo = cvt_out<YT>(acc[r][h][2 * w2][i]), hi = cvt_out<YT>(acc[r][h][2 * w2 + 1][i]);
                words[w2] = (uint32_t)__builtin_bit_cast(uint16_t, lo) | ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
              }
            }
            if constexpr (WORDS % 4 == 0) {
#pragma unroll
              for (int v = 0; v < WORDS / 4; ++v)
                ((u32x4*)dst)[v] = u32x4{words[4 * v], words[4 * v + 1], words[4 * v + 2], words[4 * v + 3]};
            } else if constexpr (WORDS == 2) {
              *(u32x2*)dst = u32x2{words[0], words[1]};
            } else {
#pragma unroll
              for (int v = 0; v < WORDS; ++v) ((uint32_t*)dst)[v] = words[v];
            }
          } else {
#pragma unroll
            for (int s = 0; s < NS; ++s)
              if (col0 + s < p.n) dst[s] = cvt_out<YT>(acc[r][h][s][i]);
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------- dispatch
template <typename XT, typename WT, typename YT, int B, int WAVES, int RW, int NS, int CW, int WCAP>
spmm_status_t launch_t(const RunArgs& a, hipStream_t stream) {
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
  p.ovf_only = a.ovf_mode == 2 ? a.ovf : nullptr;
  constexpr int NTILE = 16 * NS;
  p.ntiles = (int32_t)ceil_div(a.n, NTILE);
  const int64_t units = (int64_t)p.ntiles * a.plan.num_panels;
  if (units > (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "too many work units");
  p.num_units = (int32_t)units;
  if (units == 0) return SPMM_OK;
  if (a.gather) {
    auto k = k_spmm_mfma<XT, WT, YT, B, WAVES, RW, NS, CW, WCAP, true>;
    using Cf = Cfg<XT, WT, YT, B, WAVES, RW, NS, CW, WCAP, true>;
    SPMM_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, Cf::LDS));
    hipLaunchKernelGGL(k, dim3((unsigned)units), dim3(WAVES * 64), Cf::LDS, stream, p);
  } else {
    auto k = k_spmm_mfma<XT, WT, YT, B, WAVES, RW, NS, CW, WCAP, false>;
    using Cf = Cfg<XT, WT, YT, B, WAVES, RW, NS, CW, WCAP, false>;
    SPMM_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, Cf::LDS));
    hipLaunchKernelGGL(k, dim3((unsigned)units), dim3(WAVES * 64), Cf::LDS, stream, p);
  }
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

}  // namespace

// Variants keyed by (block size, group rows, chunk columns, dtypes). The
// group rows and chunk columns are fixed by the plan; the column tile (NS) is
// picked from n here.
template <typename XT, typename WT, typename YT>
static spmm_status_t dispatch_types(const RunArgs& a, hipStream_t s) {
  const int b = a.plan.b, GR = a.plan.group_rows, CW = a.plan.chunk_cols;
  constexpr bool F32 = __is_same(XT, float);
  const bool wide = a.n > 64;
  if (b == 16) {
    if (GR == 32 && CW == 8) {
      if constexpr (F32) return launch_t<XT, WT, YT, 16, 8, 4, 4, 8, 32>(a, s);
      else return wide ? launch_t<XT, WT, YT, 16, 8, 4, 8, 8, 64>(a, s) : launch_t<XT, WT, YT, 16, 8, 4, 4, 8, 64>(a, s);
    }
    if (GR == 8 && CW == 8) {
      if constexpr (F32) return launch_t<XT, WT, YT, 16, 4, 2, 4, 8, 16>(a, s);
      else return wide ? launch_t<XT, WT, YT, 16, 4, 2, 8, 8, 32>(a, s) : launch_t<XT, WT, YT, 16, 4, 2, 4, 8, 32>(a, s);
    }
    // geometries of the pipelined kernel (64-row chunks): general path for oversized chunks
    if constexpr (!F32) {
      if (CW == 4 && GR == 32) return launch_t<XT, WT, YT, 16, 8, 4, 4, 4, 64>(a, s);
      if (CW == 4 && GR == 16) return launch_t<XT, WT, YT, 16, 8, 2, 4, 4, 64>(a, s);
      if (CW == 4 && GR == 8) return launch_t<XT, WT, YT, 16, 4, 2, 4, 4, 64>(a, s);
    }
  } else if (b == 32) {
    if (GR == 16 && CW == 4) {
      if constexpr (F32) return launch_t<XT, WT, YT, 32, 8, 2, 4, 4, 8>(a, s);
      else return wide ? launch_t<XT, WT, YT, 32, 8, 2, 8, 4, 16>(a, s) : launch_t<XT, WT, YT, 32, 8, 2, 4, 4, 16>(a, s);
    }
    if (GR == 4 && CW == 4) {
      if constexpr (F32) return launch_t<XT, WT, YT, 32, 4, 1, 4, 4, 8>(a, s);
      else return wide ? launch_t<XT, WT, YT, 32, 4, 1, 8, 4, 16>(a, s) : launch_t<XT, WT, YT, 32, 4, 1, 4, 4, 16>(a, s);
    }
    if constexpr (!F32) {
      if (CW == 2 && GR == 16) return launch_t<XT, WT, YT, 32, 8, 2, 4, 2, 16>(a, s);
      if (CW == 2 && GR == 8) return launch_t<XT, WT, YT, 32, 4, 2, 4, 2, 16>(a, s);
    }
  }
  return fail(SPMM_ERR_UNSUPPORTED, "no MFMA kernel variant for this block size / geometry");
}

spmm_status_t launch_spmm_mfma(const RunArgs& a, hipStream_t s) {
  using spmm_bf16 = __bf16;
  if (a.wt == SPMM_F32) return dispatch_types<float, float, float>(a, s);
  if (a.wt == SPMM_F16) {
    if (a.yt == SPMM_F16) return dispatch_types<_Float16, _Float16, _Float16>(a, s);
    return dispatch_types<_Float16, _Float16, float>(a, s);
  }
  if (a.wt == SPMM_BF16) {
    if (a.yt == SPMM_BF16) return dispatch_types<spmm_bf16, spmm_bf16, spmm_bf16>(a, s);
    return dispatch_types<spmm_bf16, spmm_bf16, float>(a, s);
  }
  // FP8 weights
  if (a.xt == SPMM_F16) {
    if (a.yt == SPMM_F16) return dispatch_types<_Float16, Fp8Tag, _Float16>(a, s);
    return dispatch_types<_Float16, Fp8Tag, float>(a, s);
  }
  if (a.yt == SPMM_BF16) return dispatch_types<spmm_bf16, Fp8Tag, spmm_bf16>(a, s);
  return dispatch_types<spmm_bf16, Fp8Tag, float>(a, s);
}

}  // namespace spmm
