// Block-sparse x dense SpMM for b = 4 and 8 (and, further down, b = 1) with
// X staged in LDS and shared by a panel of block rows (PopSparse, Section 3:
// Y = (M o W) * X, FP32 accumulation; Section 3.2: the static partition of
// the known blocks).
//
// At b = 4 every block reads b rows of X for only b FLOPs per byte, so a
// kernel that reads X from L2 per block is bound by the L2 -> CU path. Here a
// workgroup owns a panel of RW x NWAVES consecutive block rows and a tile of
// 64 columns, and walks k in chunks of KC rows: the chunk of X is loaded once
// (coalesced 16-byte loads), transposed in registers and stored in LDS column
// by column (k contiguous), double-buffered so the next chunk's loads are in
// flight while the current one is used. Each wave owns RW block rows and
// consumes, per chunk, the blocks of its rows that fall in the chunk (a
// cursor per row; columns ascend inside a row, so they are a contiguous
// range).
//
// Products run on v_mfma_f32_4x4x4 (16 independent 4 x 4 x 4 products per
// instruction). Product beta takes columns 4 beta .. 4 beta + 3 of the tile,
// so lane L (beta = L / 4) supplies column L of the B operand: the 4 k values
// of its column, one 8-byte LDS read. The A operand, a 4 x 4 tile of a
// weight block, is broadcast from one product to all 16 (cbsz = 4, abid
// selects the source): lanes 4t .. 4t + 3 hold tile t of a batch of 16 tiles
// (16 blocks of b = 4, or 4 blocks of four tiles for b = 8), loaded as one
// coalesced vector load. Lane L ends up holding column L of the block row's
// 4-row output tiles.
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "common.h"

namespace spmm {
namespace {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kKC = 256;            // k rows per chunk
constexpr int kNT = 64;             // columns per tile
constexpr int kColStride = kKC + 4; // halves per LDS column (reads of 16 lanes cover the 32 banks)
constexpr int kBufHalves = kNT * kColStride;
constexpr uint32_t kOOB = 0x80000000u;
constexpr int kNW = 8;              // waves per workgroup (two workgroups share a CU's LDS)

struct LParams {
  const int32_t* row_ptr;  // [mb + 1]
  const int32_t* col_idx;  // [nnz]
  const void* W;           // block-CSR values (or indexed by w_index)
  const int32_t* w_index;  // entry q's values are block w_index[q] of W; nullptr: block q
  const void* X;
  void* Y;
  int64_t ldx, ldy;
  int32_t m, k, n, mb;
  int32_t num_units, num_panels;
  uint32_t x_bytes;        // k * ldx * 2, < 2^31
  uint32_t c_bytes, w_bytes;  // column indices and values (entries x 4 and x b * b * 2), < 2^31
  int32_t relu;
  const int32_t* status;   // skip when *status != 0 (dynamic), else nullptr
};

__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int32_t xcd_unit(int32_t w, int32_t U) {
  const int32_t q = U >> 3, r = U & 7;
  const int32_t x = w & 7, local = w >> 3;
  return x * q + min(x, r) + local;
}

// D += A x B for 16 products of 4 x 4 x 4, A broadcast from product ABID.
template <typename XT, int ABID>
__device__ __forceinline__ float4_t mma4(u32x2 a, u32x2 b, float4_t c) {
  if constexpr (__is_same(XT, _Float16))
    return __builtin_amdgcn_mfma_f32_4x4x4f16(__builtin_bit_cast(half4_t, a), __builtin_bit_cast(half4_t, b), c, 4,
                                              ABID, 0);
  else
    return __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(__builtin_bit_cast(short4_t, a), __builtin_bit_cast(short4_t, b), c,
                                                  4, ABID, 0);
}

// Workgroup barrier for the LDS pipeline: waits for this wave's LDS
// operations only (s_waitcnt lgkmcnt(0)), not for its global loads, so loads
// issued for the next chunk stay in flight across it (a full __syncthreads()
// fence would wait for them). The empty asm statements keep the compiler
// from moving memory operations across the barrier.
__device__ __forceinline__ void sync_lds() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt at their maximum (no wait)
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

template <typename YT> __device__ __forceinline__ YT to_out(float v);
template <> __device__ __forceinline__ float to_out<float>(float v) { return v; }
template <> __device__ __forceinline__ _Float16 to_out<_Float16>(float v) { return (_Float16)v; }
template <> __device__ __forceinline__ __bf16 to_out<__bf16>(float v) { return (__bf16)v; }

// Chunk staging by all NW waves of the workgroup: thread t covers columns
// 8 (t % 8) .. +8 of the tile and the row quads t / 8 + NW * 8 s: four
// 16-byte row loads per quad, transposed with v_perm into 8 columns x 4 k
// values (one 8-byte LDS store each).
template <int NW>
struct Stage {
  static constexpr int kQuads = kKC / 4;
  static constexpr int kQPT = kQuads / (NW * 8);  // quads per thread
  static_assert(kQPT * NW * 8 == kQuads, "threads must tile the chunk");
  uint32_t r[kQPT][4][4];

  __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t xr, const LParams& p, int32_t k0, int32_t n0, int pt) {
    const int cg = pt & 7;
#pragma unroll
    for (int s = 0; s < kQPT; ++s) {
      const int32_t quad = (pt >> 3) + s * NW * 8;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int32_t krow = k0 + 4 * quad + i;
        const uint32_t off = krow < p.k ? (uint32_t)(((int64_t)krow * p.ldx + n0 + 8 * cg) * 2) : kOOB;
        const u32x4 v = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(xr, off, 0, 0));
#pragma unroll
        for (int e = 0; e < 4; ++e) r[s][i][e] = v[e];
      }
    }
  }

  __device__ __forceinline__ void store(uint16_t* buf, int pt) const {
    const int cg = pt & 7;
#pragma unroll
    for (int s = 0; s < kQPT; ++s) {
      const int32_t quad = (pt >> 3) + s * NW * 8;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const uint32_t sel = (e & 1) ? 0x07060302u : 0x05040100u;
        const uint32_t lo = __builtin_amdgcn_perm(r[s][1][e >> 1], r[s][0][e >> 1], sel);
        const uint32_t hi = __builtin_amdgcn_perm(r[s][3][e >> 1], r[s][2][e >> 1], sel);
        *(u32x2*)(buf + (8 * cg + e) * kColStride + 4 * quad) = u32x2{lo, hi};
      }
    }
  }
};

// The indices and weights of a batch of up to 16 tiles of one block row
// starting at CSR entry q: lane 4t + i holds tile t's column index and row i
// of its 4 x 4 weights. Loads past the row's end are clamped to a valid entry
// and masked later, so a batch is two loads that do not wait for each other
// (three with an index map).
template <int B>
struct Batch {
  int32_t cv;  // block column of this lane's tile (0x7fffffff past the row)
  u32x2 a;     // A operand: row i of this lane's tile
};

template <int B, bool GATHER>
__device__ __forceinline__ Batch<B> load_batch(const LParams& p, __amdgpu_buffer_rsrc_t cr, __amdgpu_buffer_rsrc_t wr,
                                               int32_t q, int32_t e, int lane) {
  constexpr int TB = B / 4, TPB = TB * TB;
  const int tl = lane >> 2, ii = lane & 3;
  const int bi = tl / TPB, rt = (tl % TPB) / TB, kt = tl % TB;
  const int32_t qb = q + bi;
  const bool ok = qb < e;
  const int32_t qc = ok ? qb : max(e - 1, 0);
  Batch<B> t;
  const int32_t c = __builtin_amdgcn_raw_buffer_load_b32(cr, (uint32_t)qc * 4u, 0, 0);
  t.cv = ok ? c : 0x7fffffff;
  const uint32_t wq = GATHER ? (uint32_t)p.w_index[qc] : (uint32_t)qc;
  t.a = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(
                                      wr, (wq * (uint32_t)(B * B) + (uint32_t)((rt * 4 + ii) * B + kt * 4)) * 2u, 0, 0));
  return t;
}

// One workgroup: NW waves, each owning RW block rows of the panel and a share
// of the chunk staging; one 64-column tile; B = 4 or 8, 16-bit W and X of one
// type. Per chunk a wave (1) multiplies its rows' blocks of the chunk from LDS
// with the batches loaded during the previous chunk, (2) issues the batches
// of the next chunk, (3) stores the next chunk's X, loaded two chunks
// earlier, into the other LDS buffer, (4) issues the loads of the chunk three
// ahead. Loads complete in issue order, so every wait covers only loads
// issued at least a chunk earlier.
template <typename XT, typename YT, int B, int RW, int NW, bool GATHER>
__global__ __launch_bounds__(NW * 64) void k_spmm_small_lds(LParams p) {
  constexpr int TB = B / 4;        // row (and k) tiles of 4 per block
  constexpr int TPB = TB * TB;     // 4 x 4 tiles per block
  constexpr int BPB = 16 / TPB;    // blocks per batch of 16 tiles
  if (p.status && *p.status) return;
  extern __shared__ uint16_t lds[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = uniform(tid >> 6);
  const int32_t unit = xcd_unit(blockIdx.x, p.num_units);
  const int32_t panel = unit % p.num_panels, ntile = unit / p.num_panels;
  const int32_t n0 = ntile * kNT;
  const int32_t nch = (p.k + kKC - 1) / kKC;
  __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)p.X, (short)0, (int)p.x_bytes, 0x00020000);
  // column indices and values through 32-bit buffer offsets (sizes below 2^31 checked at launch)
  __amdgpu_buffer_rsrc_t cr = __builtin_amdgcn_make_buffer_rsrc((void*)p.col_idx, (short)0, (int)p.c_bytes, 0x00020000);
  __amdgpu_buffer_rsrc_t wr = __builtin_amdgcn_make_buffer_rsrc((void*)p.W, (short)0, (int)p.w_bytes, 0x00020000);

  const int32_t r0 = panel * (RW * NW) + wave * RW;
  int32_t cur[RW], end[RW];
#pragma unroll
  for (int i = 0; i < RW; ++i) {
    const int32_t r = min(r0 + i, p.mb);  // rows past mb: an empty range
    cur[i] = uniform(p.row_ptr[r]);
    end[i] = uniform(p.row_ptr[min(r + 1, p.mb)]);
  }
  float4_t acc[RW][TB];
#pragma unroll
  for (int i = 0; i < RW; ++i)
#pragma unroll
    for (int t = 0; t < TB; ++t) acc[i][t] = float4_t{0.f, 0.f, 0.f, 0.f};

  // Two register sets of staged X (chunks ch + 1 and ch + 2 in flight while
  // chunk ch is used from LDS); the chunk loop is unrolled by two so that
  // each set is a fixed set of registers.
  Stage<NW> sa, sb;
  Batch<B> pre[RW];  // each row's first batch of the current chunk
  sa.load(xr, p, 0, n0, tid);
  if (nch > 1) sb.load(xr, p, kKC, n0, tid);
#pragma unroll
  for (int i = 0; i < RW; ++i) pre[i] = load_batch<B, GATHER>(p, cr, wr, cur[i], end[i], lane);
  sa.store(lds, tid);
  if (nch > 2) sa.load(xr, p, 2 * kKC, n0, tid);
  sync_lds();  // chunk 0 staged

  // one chunk: multiply from LDS buffer (ch & 1), then issue the next chunk's
  // batches, store chunk ch + 1 from `nxt` and reload `nxt` with chunk ch + 3
  auto chunk = [&](int32_t ch, Stage<NW>& nxt) {
    const int32_t k0 = ch * kKC;
    const uint16_t* buf = lds + (ch & 1) * kBufHalves + lane * kColStride;
    const int32_t kend = (k0 + kKC) / B;  // first block column past the chunk
#pragma unroll
    for (int i = 0; i < RW; ++i) {
      Batch<B> bt = pre[i];
      int32_t q = cur[i];
      const int32_t e = end[i];
      for (;;) {
        const bool in = bt.cv < kend;
        // blocks of the batch inside the chunk (columns ascend: a prefix)
        const int32_t cnt = __popcll(__ballot(in && (lane & (4 * TPB - 1)) == 0));
        if (cnt == 0) break;
        const u32x2 a = in ? bt.a : u32x2{0u, 0u};
        // groups of 4 blocks: a group is skipped when no block of it is in the
        // chunk; inside a group, blocks past the chunk read a valid LDS column
        // and are masked to zero (their A tiles are zero too)
        static_for<0, BPB / 4 + (BPB < 4 ? 1 : 0)>([&](auto gg) {
          constexpr int g = decltype(gg)::value;
          constexpr int G = BPB < 4 ? BPB : 4;  // blocks per group
          if (g * G < cnt) {
            u32x2 x[G][TB];
            static_for<0, G>([&](auto jj) {
              constexpr int j = decltype(jj)::value, b = g * G + j;
              const bool live = b < cnt;
              const int32_t cl = __builtin_amdgcn_readlane(bt.cv, b * 4 * TPB);
              const int32_t c = live ? cl : k0 / B;
              const uint16_t* col = buf + (c * B - k0);
#pragma unroll
              for (int kk = 0; kk < TB; ++kk) {
                const u32x2 v = *(const u32x2*)(col + 4 * kk);
                x[j][kk] = live ? v : u32x2{0u, 0u};
              }
            });
            static_for<0, G>([&](auto jj) {
              constexpr int j = decltype(jj)::value, b = g * G + j;
              static_for<0, TPB>([&](auto tt) {
                constexpr int r = decltype(tt)::value / TB, kk = decltype(tt)::value % TB;
                acc[i][r] = mma4<XT, b * TPB + r * TB + kk>(a, x[j][kk], acc[i][r]);
              });
            });
          }
        });
        q += cnt;
        if (cnt < BPB || q >= e) break;
        bt = load_batch<B, GATHER>(p, cr, wr, q, e, lane);  // a row with more blocks in this chunk than one batch
      }
      cur[i] = q;
    }
    if (ch + 1 < nch) {
#pragma unroll
      for (int i = 0; i < RW; ++i) pre[i] = load_batch<B, GATHER>(p, cr, wr, cur[i], end[i], lane);
      nxt.store(lds + ((ch + 1) & 1) * kBufHalves, tid);
      if (ch + 3 < nch) nxt.load(xr, p, (ch + 3) * kKC, n0, tid);
    }
    sync_lds();  // chunk ch consumed; chunk ch + 1 staged
  };
  for (int32_t ch = 0; ch < nch; ch += 2) {
    chunk(ch, sb);                     // chunk 1 (then 3, ...) waits in set b
    if (ch + 1 < nch) chunk(ch + 1, sa);  // chunk 2 (then 4, ...) in set a
  }

  // lane L holds column n0 + L of rows 4 t + j (j = 0..3) of each block row
  const int32_t col = n0 + lane;
  if (col >= p.n) return;
  YT* __restrict__ Y = (YT*)p.Y;
#pragma unroll
  for (int i = 0; i < RW; ++i) {
    const int32_t r = r0 + i;
    if (r >= p.mb) break;
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t row = (int64_t)r * B + 4 * t + j;
        if (row >= p.m) continue;
        float v = acc[i][t][j];
        if (p.relu) v = v > 0.f ? v : 0.f;
        Y[row * p.ldy + col] = to_out<YT>(v);
      }
  }
}

template <typename XT, typename YT, int B, int RW, int NW, bool GATHER>
spmm_status_t launch_lds(const RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx, hipStream_t s) {
  LParams p;
  p.row_ptr = row_ptr;
  p.col_idx = col_idx;
  p.W = a.W;
  p.w_index = a.w_index;
  p.X = a.X;
  p.Y = a.Y;
  p.ldx = a.ldx;
  p.ldy = a.ldy;
  p.m = a.plan.m;
  p.k = a.plan.k;
  p.n = a.n;
  p.mb = a.plan.mb;
  p.relu = a.relu ? 1 : 0;
  p.status = a.status;
  const int64_t xb = (int64_t)a.plan.k * a.ldx * 2;
  if (xb >= (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "X larger than 2 GiB is not supported");
  p.x_bytes = (uint32_t)xb;
  const int64_t cb = a.nnz * 4, wb = a.nnz * (int64_t)B * B * 2;
  if (cb >= (int64_t)INT32_MAX || wb >= (int64_t)INT32_MAX)
    return fail(SPMM_ERR_UNSUPPORTED, "more than 2 GiB of values is not supported");
  p.c_bytes = (uint32_t)std::max<int64_t>(cb, 4);
  p.w_bytes = (uint32_t)std::max<int64_t>(wb, 4);
  const int64_t panels = ceil_div(a.plan.mb, (int64_t)RW * NW);
  const int64_t units = panels * ceil_div(a.n, kNT);
  if (units == 0) return SPMM_OK;
  if (units > (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "too many work units");
  p.num_panels = (int32_t)panels;
  p.num_units = (int32_t)units;
  const size_t lds = 2 * (size_t)kBufHalves * sizeof(uint16_t);
  static const hipError_t attr = hipFuncSetAttribute((const void*)k_spmm_small_lds<XT, YT, B, RW, NW, GATHER>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return fail_hip(attr, "LDS limit of the small-block kernel");
  hipLaunchKernelGGL((k_spmm_small_lds<XT, YT, B, RW, NW, GATHER>), dim3((unsigned)units), dim3(NW * 64), lds, s, p);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

// Rows per wave: the most that still give the launch about two workgroups per
// CU (fewer rows per panel share each staged chunk among fewer blocks).
template <typename XT, typename YT, int B>
spmm_status_t small_lds_b(const RunArgs& a, const int32_t* rp, const int32_t* ci, hipStream_t s, int rw) {
  constexpr int R0 = 8;
  // static plans keep their values in CSR order; dynamic calls read them through an index map
  if (a.w_index) {
    if (rw >= R0) return launch_lds<XT, YT, B, R0, kNW, true>(a, rp, ci, s);
    if (rw >= R0 / 2) return launch_lds<XT, YT, B, R0 / 2, kNW, true>(a, rp, ci, s);
    return launch_lds<XT, YT, B, R0 / 4, kNW, true>(a, rp, ci, s);
  }
  if (rw >= R0) return launch_lds<XT, YT, B, R0, kNW, false>(a, rp, ci, s);
  if (rw >= R0 / 2) return launch_lds<XT, YT, B, R0 / 2, kNW, false>(a, rp, ci, s);
  return launch_lds<XT, YT, B, R0 / 4, kNW, false>(a, rp, ci, s);
}

template <typename XT, typename YT>
spmm_status_t small_lds_y(const RunArgs& a, const int32_t* rp, const int32_t* ci, hipStream_t s, int rw) {
  if (a.plan.b == 8) return small_lds_b<XT, YT, 8>(a, rp, ci, s, rw);
  return small_lds_b<XT, YT, 4>(a, rp, ci, s, rw);
}

// ------------------------------------------------------------------ b = 1
// Unstructured sparsity (b = 1) with X staged in LDS. The kernel without LDS
// reads one X row from L2 per nonzero: 2 bytes per FMA, which binds it to
// the L1 -> L2 path. Here a workgroup of NW waves owns a panel of RW x NW
// rows and a tile of 512 columns, and walks k in chunks of KC rows: the
// chunk (KC x 512 values) is loaded once, one k row per wave instruction,
// and stored row-major in LDS (two buffers; two register sets of chunk loads
// in flight, each chunk loaded three chunks ahead). Each wave owns RW rows and takes, per chunk, the nonzeros of
// each row that fall in the chunk (a cursor per row: columns ascend, so
// they are the next entries of the row). Lane L covers columns 8L .. 8L + 7
// of the tile: per nonzero one 16-byte LDS read; the FMAs run on v_dot2
// over two nonzeros of the row (their two X values interleaved with v_perm,
// their two weights packed in one dword), FP32 accumulation. Rows go in
// pairs, two slots of each at a time; slots past a row's nonzeros read an
// LDS row of zeros with weight 0. Traffic from L2 per panel is the chunk
// loads, 2 / (RW x NW x density) bytes per FMA.
// V values (8 or 4) of 16 bits as dwords: one lane's share of an X row.
template <int V>
struct XSeg {
  static_assert(V == 8 || V == 4, "8 or 4 columns per lane");
  uint32_t d[V / 2];
  __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t xr, uint32_t off) {
    if constexpr (V == 8) {
      const u32x4 v = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(xr, off, 0, 0));
#pragma unroll
      for (int i = 0; i < 4; ++i) d[i] = v[i];
    } else {
      const u32x2 v = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(xr, off, 0, 0));
      d[0] = v.x;
      d[1] = v.y;
    }
  }
  __device__ __forceinline__ void read(const uint16_t* a) {
    if constexpr (V == 8) {
      const u32x4 v = *(const u32x4*)a;
#pragma unroll
      for (int i = 0; i < 4; ++i) d[i] = v[i];
    } else {
      const u32x2 v = *(const u32x2*)a;
      d[0] = v.x;
      d[1] = v.y;
    }
  }
  __device__ __forceinline__ void write(uint16_t* a) const {
    if constexpr (V == 8) *(u32x4*)a = u32x4{d[0], d[1], d[2], d[3]};
    else *(u32x2*)a = u32x2{d[0], d[1]};
  }
};

template <int KC, int NW, int V>
struct Stage1 {
  static constexpr int NT = 64 * V;      // columns per tile
  static constexpr int kRows = KC / NW;  // k rows per wave
  static_assert(kRows * NW == KC, "waves must tile the chunk");
  XSeg<V> r[kRows];

  __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t xr, const LParams& p, int32_t k0, int32_t n0, int wave,
                                       int lane) {
#pragma unroll
    for (int s = 0; s < kRows; ++s) {
      const int32_t krow = k0 + wave + s * NW;
      const uint32_t off = krow < p.k ? (uint32_t)(((int64_t)krow * p.ldx + n0 + V * lane) * 2) : kOOB;
      r[s].load(xr, off);
    }
  }

  __device__ __forceinline__ void store(uint16_t* buf, int wave, int lane) const {
#pragma unroll
    for (int s = 0; s < kRows; ++s) r[s].write(buf + (wave + s * NW) * NT + V * lane);
  }
};

// 64 entries of one row starting at CSR entry q, one per lane: column index
// and 16-bit weight bits. Lanes past the row's end e load from an offset past
// the buffer (zero, no memory access); they are masked out of the ballot by
// valid_lanes(e - q) where the batch is used. Nothing is computed from the
// loaded values here, so the loads stay in flight until their first use.
struct Batch1 {
  int32_t cv;
  uint32_t wv;
};

template <bool GATHER>
__device__ __forceinline__ Batch1 load_batch1(__amdgpu_buffer_rsrc_t cr, __amdgpu_buffer_rsrc_t wr,
                                              __amdgpu_buffer_rsrc_t ir, int32_t q, int32_t e, int lane) {
  const int32_t qb = q + lane;
  const uint32_t off = qb < e ? (uint32_t)qb * 4u : kOOB;
  Batch1 t;
  t.cv = __builtin_amdgcn_raw_buffer_load_b32(cr, off, 0, 0);
  if constexpr (GATHER) {
    const uint32_t wq = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(ir, off, 0, 0);
    t.wv = __builtin_amdgcn_raw_buffer_load_b16(wr, qb < e ? wq * 2u : kOOB, 0, 0);
  } else {
    t.wv = __builtin_amdgcn_raw_buffer_load_b16(wr, qb < e ? (uint32_t)qb * 2u : kOOB, 0, 0);
  }
  return t;
}

// Lanes 0 .. d - 1 of a batch hold entries of the row (d = entries left).
__device__ __forceinline__ uint64_t valid_lanes(int32_t d) {
  return d >= 64 ? ~0ull : (d <= 0 ? 0ull : (1ull << d) - 1ull);
}

template <typename XT> struct Dot2;
template <> struct Dot2<_Float16> {
  static __device__ __forceinline__ float f(uint32_t a, uint32_t b, float c) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    return __builtin_amdgcn_fdot2(__builtin_bit_cast(h2, a), __builtin_bit_cast(h2, b), c, false);
  }
};
template <> struct Dot2<__bf16> {
  static __device__ __forceinline__ float f(uint32_t a, uint32_t b, float c) {
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(b2, a), __builtin_bit_cast(b2, b), c, false);
  }
};

// A batch's entries as one dword per lane: weight bits << 16 | column - k0
// (the column's row in the staged chunk) for the lanes in `live`; the other
// lanes get weight 0 and row KC, an LDS row of zeros, so that any group of
// slots can be processed without masks.
template <int KC>
__device__ __forceinline__ uint32_t pack_batch(const Batch1& bt, int32_t k0, uint64_t live, int lane) {
  const bool on = (live >> lane) & 1ull;
  return on ? (bt.wv << 16) | ((uint32_t)(bt.cv - k0) & 0xFFFFu) : (uint32_t)KC;
}

// Slots t .. t + S - 1 of a packed batch (S = 2 or 4; slots past a row's
// nonzeros read the zero row with weight 0). `row` is this lane's part of
// LDS row 0 of the chunk.
template <typename XT, int V, int S>
__device__ __forceinline__ void b1_group(float (&acc)[V], uint32_t pk, int32_t t, const uint16_t* row) {
  static_assert(S == 2 || S == 4, "slots in pairs");
  uint32_t w[S];
  XSeg<V> x[S];
#pragma unroll
  for (int j = 0; j < S; ++j) {
    const uint32_t e = (uint32_t)__builtin_amdgcn_readlane((int)pk, t + j);
    w[j] = e >> 16;
    x[j].read(row + (e & 0xFFFFu) * (64 * V));
  }
#pragma unroll
  for (int pr = 0; pr < S / 2; ++pr) {
    const uint32_t wp = w[2 * pr] | (w[2 * pr + 1] << 16);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const uint32_t sel = (v & 1) ? 0x07060302u : 0x05040100u;
      const uint32_t xp = __builtin_amdgcn_perm(x[2 * pr + 1].d[v >> 1], x[2 * pr].d[v >> 1], sel);
      acc[v] = Dot2<XT>::f(wp, xp, acc[v]);
    }
  }
}

template <typename XT, typename YT, int RW, int NW, int KC, int V, int MINB, bool GATHER>
__global__ __launch_bounds__(NW * 64, MINB) void k_spmm_b1_lds(LParams p) {
  constexpr int NT = 64 * V;
  if (p.status && *p.status) return;
  extern __shared__ uint16_t lds[];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = uniform(tid >> 6);
  const int32_t unit = xcd_unit(blockIdx.x, p.num_units);
  const int32_t panel = unit % p.num_panels, ntile = unit / p.num_panels;
  const int32_t n0 = ntile * NT;
  const int32_t nch = (p.k + KC - 1) / KC;
  __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)p.X, (short)0, (int)p.x_bytes, 0x00020000);
  __amdgpu_buffer_rsrc_t cr = __builtin_amdgcn_make_buffer_rsrc((void*)p.col_idx, (short)0, (int)p.c_bytes, 0x00020000);
  __amdgpu_buffer_rsrc_t wr = __builtin_amdgcn_make_buffer_rsrc((void*)p.W, (short)0, (int)p.w_bytes, 0x00020000);
  // the index map of dynamic calls, as large as the column indices
  __amdgpu_buffer_rsrc_t ir =
      __builtin_amdgcn_make_buffer_rsrc((void*)p.w_index, (short)0, GATHER ? (int)p.c_bytes : 0, 0x00020000);

  const int32_t r0 = panel * (RW * NW) + wave * RW;
  int32_t cur[RW], end[RW];
#pragma unroll
  for (int i = 0; i < RW; ++i) {
    const int32_t r = min(r0 + i, p.mb);  // rows past mb: an empty range
    cur[i] = uniform(p.row_ptr[r]);
    end[i] = uniform(p.row_ptr[min(r + 1, p.mb)]);
  }
  float acc[RW][V];
#pragma unroll
  for (int i = 0; i < RW; ++i)
#pragma unroll
    for (int v = 0; v < V; ++v) acc[i][v] = 0.f;

  // A row holds at most one entry per column, so with KC <= 64 one batch of
  // 64 lanes holds all of a row's entries in a chunk. Dynamic calls may hold
  // duplicates (summed): there a row can run past its batch, and the code
  // for that (DUP) reloads it.
  static_assert(KC <= 64, "a chunk's entries of a row fit one batch");
  static_assert(RW % 2 == 0, "rows are multiplied in pairs");
  constexpr int SL = 2;  // slots per row per step of the pair loop
  constexpr bool DUP = GATHER;
  constexpr int BUF = (KC + 1) * NT;  // halves per LDS buffer: KC rows of X and a row of zeros
  Batch1 bt[RW];   // each row's entries from position bq (loaded one chunk ahead)
  int32_t bq[RW];
  // Two register sets of X in flight: chunk c is loaded during chunk c - 3
  // (or the prologue), stored into LDS at the start of chunk c - 1 and used in
  // chunk c. Loads past the last chunk read zeros (offsets past the buffer),
  // so every load and store is unconditional and each wait is a count of
  // loads issued later (loads complete in issue order).
  Stage1<KC, NW, V> sa, sb;
  sb.load(xr, p, 0, n0, wave, lane);
#pragma unroll
  for (int i = 0; i < RW; ++i) {
    bt[i] = load_batch1<GATHER>(cr, wr, ir, cur[i], end[i], lane);
    bq[i] = cur[i];
  }
  if (wave == 0) {
    XSeg<V> z;
#pragma unroll
    for (int i = 0; i < V / 2; ++i) z.d[i] = 0u;
    z.write(lds + KC * NT + V * lane);
    z.write(lds + BUF + KC * NT + V * lane);
  }
  sb.store(lds, wave, lane);
  sa.load(xr, p, KC, n0, wave, lane);
  sb.load(xr, p, 2 * KC, n0, wave, lane);
  sync_lds();  // chunk 0 staged; chunks 1 and 2 in flight

  // One chunk: (1) store chunk ch + 1 from `nxt` into the other LDS buffer,
  // count each row's entries inside chunk ch and pack its batch; (2) load
  // chunk ch + 3 into `nxt` and the next chunk's batches; (3) multiply from
  // LDS, two rows at a time (their LDS reads in flight together); a barrier.
  auto chunk = [&](int32_t ch, Stage1<KC, NW, V>& nxt) {
    const int32_t k0 = ch * KC, kend = k0 + KC;
    nxt.store(lds + ((ch + 1) & 1) * BUF, wave, lane);
    uint32_t pk[RW];
    int32_t cnt[RW];
#pragma unroll
    for (int i = 0; i < RW; ++i) {
      if constexpr (DUP) {
        if (bq[i] != cur[i]) {  // the row ran past its batch in the previous chunk
          bt[i] = load_batch1<GATHER>(cr, wr, ir, cur[i], end[i], lane);
          bq[i] = cur[i];
        }
      }
      // entries of the batch inside the chunk (columns ascend: a prefix)
      const uint64_t live = __ballot(bt[i].cv < kend) & valid_lanes(end[i] - cur[i]);
      cnt[i] = __popcll(live);
      pk[i] = pack_batch<KC>(bt[i], k0, live, lane);
    }
#pragma unroll
    for (int i = 0; i < RW; ++i) {
      bq[i] = cur[i] + cnt[i];
      bt[i] = load_batch1<GATHER>(cr, wr, ir, bq[i], end[i], lane);
    }
    nxt.load(xr, p, k0 + 3 * KC, n0, wave, lane);
    const uint16_t* row = lds + (ch & 1) * BUF + V * lane;
#pragma unroll
    for (int i = 0; i < RW; i += 2) {
      const int32_t nt = max(cnt[i], cnt[i + 1]);
      for (int32_t t = 0; t < nt; t += SL) {
        b1_group<XT, V, SL>(acc[i], pk[i], t, row);
        b1_group<XT, V, SL>(acc[i + 1], pk[i + 1], t, row);
      }
    }
#pragma unroll
    for (int i = 0; i < RW; ++i) {
      int32_t q = cur[i] + cnt[i];
      if constexpr (DUP) {
        if (cnt[i] == 64 && q < end[i]) {
          for (;;) {
            const Batch1 x = load_batch1<GATHER>(cr, wr, ir, q, end[i], lane);
            const uint64_t live = __ballot(x.cv < kend) & valid_lanes(end[i] - q);
            const int32_t c = __popcll(live);
            if (c == 0) break;
            const uint32_t xp = pack_batch<KC>(x, k0, live, lane);
            for (int32_t t = 0; t < c; t += 4) b1_group<XT, V, 4>(acc[i], xp, t, row);
            q += c;
            if (c < 64 || q >= end[i]) break;
          }
        }
      }
      cur[i] = q;
    }
    sync_lds();  // chunk ch consumed; chunk ch + 1 staged
  };
  // an even number of chunks (the one past k, if any, has no entries), so
  // that both halves of the loop body always run
  for (int32_t ch = 0; ch < nch; ch += 2) {
    chunk(ch, sa);      // chunk 1 (then 3, ...) waits in set a
    chunk(ch + 1, sb);  // chunk 2 (then 4, ...) in set b
  }

  // lane holds columns n0 + V lane .. + V - 1 of rows r0 .. r0 + RW - 1
  const int32_t col0 = n0 + V * lane;
  if (col0 >= p.n) return;
  YT* __restrict__ Y = (YT*)p.Y;
#pragma unroll
  for (int i = 0; i < RW; ++i) {
    const int32_t r = r0 + i;
    if (r >= p.m) break;
    float v[V];
#pragma unroll
    for (int e = 0; e < V; ++e) v[e] = p.relu ? (acc[i][e] > 0.f ? acc[i][e] : 0.f) : acc[i][e];
    YT* dst = Y + (int64_t)r * p.ldy + col0;
    if (col0 + V <= p.n) {
      if constexpr (sizeof(YT) == 4) {
#pragma unroll
        for (int e = 0; e < V; e += 4) *(float4_t*)(dst + e) = float4_t{v[e], v[e + 1], v[e + 2], v[e + 3]};
      } else {
        XSeg<V> o;
#pragma unroll
        for (int e = 0; e < V / 2; ++e)
          o.d[e] = (uint32_t)__builtin_bit_cast(uint16_t, to_out<YT>(v[2 * e])) |
                   ((uint32_t)__builtin_bit_cast(uint16_t, to_out<YT>(v[2 * e + 1])) << 16);
        o.write((uint16_t*)dst);
      }
    } else {
#pragma unroll
      for (int e = 0; e < V; ++e)
        if (col0 + e < p.n) dst[e] = to_out<YT>(v[e]);
    }
  }
}

template <typename XT, typename YT, int RW, int NW, int KC, int V, bool GATHER>
spmm_status_t launch_b1(const RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx, hipStream_t s) {
  LParams p;
  p.row_ptr = row_ptr;
  p.col_idx = col_idx;
  p.W = a.W;
  p.w_index = a.w_index;
  p.X = a.X;
  p.Y = a.Y;
  p.ldx = a.ldx;
  p.ldy = a.ldy;
  p.m = a.plan.m;
  p.k = a.plan.k;
  p.n = a.n;
  p.mb = a.plan.mb;
  p.relu = a.relu ? 1 : 0;
  p.status = a.status;
  const int64_t xb = (int64_t)a.plan.k * a.ldx * 2;
  if (xb >= (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "X larger than 2 GiB is not supported");
  p.x_bytes = (uint32_t)xb;
  const int64_t cb = a.nnz * 4, wb = a.nnz * 2;
  if (cb >= (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "more than 2 GiB of indices is not supported");
  p.c_bytes = (uint32_t)std::max<int64_t>(cb, 4);
  p.w_bytes = (uint32_t)std::max<int64_t>(wb, 4);
  const int64_t panels = ceil_div(a.plan.mb, (int64_t)RW * NW);
  const int64_t units = panels * ceil_div(a.n, 64 * V);
  if (units == 0) return SPMM_OK;
  if (units > (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "too many work units");
  p.num_panels = (int32_t)panels;
  p.num_units = (int32_t)units;
  constexpr size_t lds = 2 * (size_t)(KC + 1) * 64 * V * sizeof(uint16_t);
  constexpr int MINB = lds <= 80 * 1024 ? 2 : 1;  // workgroups per CU the LDS allows
  static const hipError_t attr = hipFuncSetAttribute((const void*)k_spmm_b1_lds<XT, YT, RW, NW, KC, V, MINB, GATHER>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return fail_hip(attr, "LDS limit of the b = 1 kernel");
  hipLaunchKernelGGL((k_spmm_b1_lds<XT, YT, RW, NW, KC, V, MINB, GATHER>), dim3((unsigned)units), dim3(NW * 64), lds, s,
                     p);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

template <typename XT, typename YT, int KC, int V>
spmm_status_t b1_lds_cfg(const RunArgs& a, const int32_t* rp, const int32_t* ci, hipStream_t s, int rw) {
  if (a.w_index) {
    if (rw >= 8) return launch_b1<XT, YT, 8, kNW, KC, V, true>(a, rp, ci, s);
    return launch_b1<XT, YT, 4, kNW, KC, V, true>(a, rp, ci, s);
  }
  if (rw >= 8) return launch_b1<XT, YT, 8, kNW, KC, V, false>(a, rp, ci, s);
  return launch_b1<XT, YT, 4, kNW, KC, V, false>(a, rp, ci, s);
}

template <typename XT, typename YT>
spmm_status_t b1_lds_y(const RunArgs& a, const int32_t* rp, const int32_t* ci, hipStream_t s, int rw) {
  return b1_lds_cfg<XT, YT, 64, 8>(a, rp, ci, s, rw);
}

}  // namespace

// Measured on MI355X at m = k = 8192 (FP16). For both block sizes the
// crossover falls with n: without LDS every block reads its X rows from L2,
// and at large n X no longer stays there. Below the crossover a panel's
// nonzeros are too few to pay for staging every chunk of X and the per-row,
// per-chunk work. b = 4, LDS against no LDS: n = 16384, 3.25 against 6.35
// ms at 1/8 and 2.46 against 3.33 ms at 1/16 (at 1/32, 2.08 against 1.74
// ms: slower); n = 4096, 85 against 74 TFLOP/s at 1/8, 95 against 77 at 1/4,
// slower at 1/16 (and at n = 8192, 1.29 against 1.25 ms); n = 1024, 0.239
// against 0.259 ms at 1/8; n = 256, 0.133 against 0.116 ms at 1/4 (slower).
// b = 1, LDS against no LDS: n =
// 16384, 8.9 against 13.2 ms at 1/16 (at 1/32, 7.1 against 6.7 ms: slower);
// n = 4096 and 8192, 3.27 against 3.59 and 6.58 against 7.64 ms at 1/8
// (losing at 1/16); n = 1024 and 2048, 1.32 against 1.39 and 2.60 against
// 2.99 ms at 1/4 (losing at 1/8); at n <= 512, where most lanes of its
// 512-column tiles idle, it loses at every density. b = 8 (the b = 4 kernel
// with four 4 x 4 tiles per block): slower than the kernel without LDS at
// every point measured, once that kernel orders its units by row slices at
// large n (n = 16384: 2.90 against 2.17 ms at 1/8, 1.93 against 1.23 ms at
// 1/16; n = 4096: 0.77 against 0.44 ms at 1/8), so the rule never takes it;
// the tuner still times it. The n = 16384 figures for b = 4 and 1 above
// are against the kernel without LDS in row-first order; with row slices it
// takes 2.60 and 4.57 ms for b = 4 (1/16, 1/8) and 12.4 and 24.1 ms for
// b = 1 (1/16, 1/8), so the LDS kernels still win there. SPMM_SMALL_LDS=0 /
// 1 forces the choice (for comparisons and tests).
bool small_lds_eligible(int32_t b, spmm_dtype_t w, spmm_dtype_t x) {
  return (b == 1 || b == 4 || b == 8) && w == x && (x == SPMM_F16 || x == SPMM_BF16);
}

bool small_lds_preferred(int32_t b, spmm_dtype_t w, spmm_dtype_t x, int64_t nnz, int64_t mb, int64_t kb, int64_t n) {
  if (!small_lds_eligible(b, w, x)) return false;
  if (const char* e = getenv("SPMM_SMALL_LDS")) {
    if (e[0] == '0') return false;
    if (e[0] == '1') return true;
  }
  // the least density (as 1 / inv) at which the LDS kernel wins, by n
  const int64_t inv = b == 1   ? (n >= 16384 ? 16 : n >= 4096 ? 8 : n >= 1024 ? 4 : 0)
                      : b == 4 ? (n >= 16384 ? 16 : n >= 1024 ? 8 : 0)
                               : 0;
  return inv > 0 && nnz * inv >= mb * kb;
}

int32_t small_lds_rows_per_wave(int32_t b, int32_t mb, int64_t n, int num_cus) {
  const int32_t r0 = 8;
  if (const char* e = getenv("SPMM_LDS_RW")) {  // tuning override
    const int v = atoi(e);
    if (v == r0 || v == r0 / 2 || v == r0 / 4) return v;
  }
  if (b == 1) return ceil_div(mb, (int64_t)r0 * kNW) * ceil_div(n, 512) >= (int64_t)num_cus ? r0 : r0 / 2;
  const int64_t tiles = ceil_div(n, kNT);
  for (int32_t rw = r0; rw > r0 / 4; rw /= 2)
    if (ceil_div(mb, (int64_t)rw * kNW) * tiles >= 2 * (int64_t)num_cus) return rw;
  return r0 / 4;
}

spmm_status_t launch_spmm_small_lds(const RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx, int32_t rw,
                                    hipStream_t s) {
  if (a.plan.b != 1 && a.plan.b != 4 && a.plan.b != 8)
    return fail(SPMM_ERR_UNSUPPORTED, "LDS small-block kernel: b = 1, 4 or 8");
  if (a.wt != a.xt || (a.xt != SPMM_F16 && a.xt != SPMM_BF16))
    return fail(SPMM_ERR_UNSUPPORTED, "LDS small-block kernel: 16-bit W and X of one type");
  if (a.plan.b == 1) {
    if (a.xt == SPMM_F16) {
      if (a.yt == SPMM_F32) return b1_lds_y<_Float16, float>(a, row_ptr, col_idx, s, rw);
      return b1_lds_y<_Float16, _Float16>(a, row_ptr, col_idx, s, rw);
    }
    if (a.yt == SPMM_F32) return b1_lds_y<__bf16, float>(a, row_ptr, col_idx, s, rw);
    return b1_lds_y<__bf16, __bf16>(a, row_ptr, col_idx, s, rw);
  }
  if (a.xt == SPMM_F16) {
    if (a.yt == SPMM_F32) return small_lds_y<_Float16, float>(a, row_ptr, col_idx, s, rw);
    return small_lds_y<_Float16, _Float16>(a, row_ptr, col_idx, s, rw);
  }
  if (a.yt == SPMM_F32) return small_lds_y<__bf16, float>(a, row_ptr, col_idx, s, rw);
  return small_lds_y<__bf16, __bf16>(a, row_ptr, col_idx, s, rw);
}

}  // namespace spmm
