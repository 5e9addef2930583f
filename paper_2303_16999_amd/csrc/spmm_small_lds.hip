// Block-sparse x dense SpMM for b = 4 with X staged in LDS and shared
// by a panel of block rows (PopSparse, Section 3: Y = (M o W) * X, FP32
// accumulation; Section 3.2: the static partition of the known blocks).
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
  return small_lds_b<XT, YT, 4>(a, rp, ci, s, rw);
}

}  // namespace

// Measured on MI355X at m = k = 8192 (FP16): the LDS kernel is faster at
// b = 4 from density 1/8 up (n = 4096: 85 against 74 TFLOP/s at 1/8, 95
// against 77 at 1/4) and slower below, where a panel's blocks are too few to
// pay for staging every chunk of X and the per-row, per-chunk work; at b = 8
// the kernel without LDS was faster at every density. SPMM_SMALL_LDS=0 / 1
// forces the choice (for comparisons and tests).
bool small_lds_eligible(int32_t b, spmm_dtype_t w, spmm_dtype_t x) {
  return b == 4 && w == x && (x == SPMM_F16 || x == SPMM_BF16);
}

bool small_lds_preferred(int32_t b, spmm_dtype_t w, spmm_dtype_t x, int64_t nnz, int64_t mb, int64_t kb) {
  if (!small_lds_eligible(b, w, x)) return false;
  if (const char* e = getenv("SPMM_SMALL_LDS")) {
    if (e[0] == '0') return false;
    if (e[0] == '1') return true;
  }
  return nnz * 8 >= mb * kb;
}

int32_t small_lds_rows_per_wave(int32_t b, int32_t mb, int64_t n, int num_cus) {
  const int32_t r0 = 8;
  if (const char* e = getenv("SPMM_LDS_RW")) {  // tuning override
    const int v = atoi(e);
    if (v == r0 || v == r0 / 2 || v == r0 / 4) return v;
  }
  const int64_t tiles = ceil_div(n, kNT);
  for (int32_t rw = r0; rw > r0 / 4; rw /= 2)
    if (ceil_div(mb, (int64_t)rw * kNW) * tiles >= 2 * (int64_t)num_cus) return rw;
  return r0 / 4;
}

spmm_status_t launch_spmm_small_lds(const RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx, int32_t rw,
                                    hipStream_t s) {
  if (a.plan.b != 4) return fail(SPMM_ERR_UNSUPPORTED, "LDS small-block kernel: b = 4");
  if (a.wt != a.xt || (a.xt != SPMM_F16 && a.xt != SPMM_BF16))
    return fail(SPMM_ERR_UNSUPPORTED, "LDS small-block kernel: 16-bit W and X of one type");
  if (a.xt == SPMM_F16) {
    if (a.yt == SPMM_F32) return small_lds_y<_Float16, float>(a, row_ptr, col_idx, s, rw);
    return small_lds_y<_Float16, _Float16>(a, row_ptr, col_idx, s, rw);
  }
  if (a.yt == SPMM_F32) return small_lds_y<__bf16, float>(a, row_ptr, col_idx, s, rw);
  return small_lds_y<__bf16, __bf16>(a, row_ptr, col_idx, s, rw);
}

}  // namespace spmm
