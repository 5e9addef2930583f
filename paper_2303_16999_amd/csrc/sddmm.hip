// Block-sampled dense-dense product (SDDMM): the weight gradient of the
// block-sparse SpMM, G_rc = dY[rows of r] * X[rows of c]^T for every nonzero
// block (r, c) of a plan (the derivative of Y = (M o W) X with respect to the
// kept weights; PopSparse, Sections 1 and 3).
//
// A task is (block row r, up to a fixed number of consecutive blocks of that
// row in CSR order). With few tasks, one runs on a workgroup of 4 waves and
// the reduction over n, in steps of 64 (two 16x16x32 MFMAs), is cut into 4
// contiguous ranges, one per wave; with many, each wave runs a task over all
// of n.
// The A operand is 16 rows of dY (lane (g, i): 8 consecutive n values of row
// i, one 16-byte load), the B operand 16 rows of X (lane (g, j): 8 n values of
// row j), so no transpose is needed; the A fragment is reused by all of the
// task's blocks, and each wave loads the next step's fragments before the
// MFMAs of the current one. Split partial sums meet in LDS and are added in
// wave order, so the result does not depend on timing. b = 32 blocks are
// 2 x 2 tiles of 16. For b = 1, 4 and 8 one MFMA computes 16 / b blocks of
// the row at once: A holds the b rows of dY (rows b .. 15 zero), B the b rows
// of X of each of the 16 / b blocks side by side, and the first b rows of the
// 16 x 16 result are those blocks; the MFMA does more arithmetic than needed,
// but the product is bound by its loads, which carry no padding.
// Rows past m or k read as zero (buffer loads), and n values past n are zeroed
// in registers, so edge blocks come out zero outside the matrix.
// G is FP32, [nnzb][b][b] row-major, in the plan's CSR order.
#include "common.h"

namespace spmm {
namespace {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr uint32_t kOOB = 0x80000000u;
// MFMA column groups per task: 4 for b = 16 (8 measured no faster: the dY
// fragment's reuse gains less than the halved occupancy costs), 2 for b = 32
// (16% faster than 1 at m = k = 8192, n = 4096, d = 1/16), 4 for b < 16.
template <int B>
__host__ __device__ constexpr int task_groups() { return B == 32 ? 2 : 4; }
// Blocks of one MFMA column group: 16 / b for b < 16, else one.
template <int B>
__host__ __device__ constexpr int group_blocks() { return B < 16 ? 16 / B : 1; }
// Blocks of one row per task.
template <int B>
__host__ __device__ constexpr int task_blocks() { return task_groups<B>() * group_blocks<B>(); }

struct SddmmParams {
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const int32_t* tasks;  // [num_tasks][2]: block row, first CSR entry
  int32_t num_tasks;
  const void* dY;
  const void* X;
  float* G;
  int64_t lddy, ldx;
  int32_t m, k, n;
  uint32_t dy_bytes, x_bytes;
};

template <typename T> struct Mfma;
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

__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// 8 consecutive 16-bit values of row `row` starting at column c0 (zero past
// `rows` via the buffer bounds, and past column n by masking).
__device__ __forceinline__ u32x4 load8(__amdgpu_buffer_rsrc_t rsrc, int64_t row, int32_t rows, int64_t ld, int32_t c0,
                                       int32_t n) {
  const uint32_t off = row < rows ? (uint32_t)((row * ld + c0) * 2) : kOOB;
  u32x4 v = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, off, 0, 0));
  const int32_t valid = n - c0;  // values of this lane inside [0, n)
  if (valid < 8) {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int32_t lo = 2 * d, hi = 2 * d + 1;
      uint32_t w = v[d];
      if (hi >= valid) w &= 0x0000FFFFu;
      if (lo >= valid) w = 0u;
      v[d] = w;
    }
  }
  return v;
}

// Wave-uniform load of an index array that no kernel writes while it runs
// (constant address space: a scalar load).
__device__ __forceinline__ int32_t sload(const int32_t* base, int64_t i) {
  typedef const __attribute__((address_space(4))) int32_t* cptr;
  return uniform(((cptr)base)[i]);
}

__device__ __forceinline__ int32_t xcd_task(int32_t w, int32_t U) {
  // consecutive tasks (often one block row, so the same dY rows) on one XCD
  const int32_t q = U >> 3, r = U & 7;
  const int32_t x = w & 7, local = w >> 3;
  return x * q + min(x, r) + local;
}

template <int B>
__host__ __device__ constexpr int tiles() { return B < 16 ? 1 : B / 16; }

template <int B>
__host__ __device__ constexpr int sddmm_lds_bytes() {
  return 4 * task_groups<B>() * tiles<B>() * tiles<B>() * 64 * 16;
}

template <typename T, int B, bool SPLIT>
__global__ __launch_bounds__(256) void k_sddmm(SddmmParams p) {
  constexpr int H = tiles<B>();
  constexpr int G = task_groups<B>();   // MFMA column groups per task
  constexpr int BG = group_blocks<B>();  // blocks per group
  constexpr bool kSmall = B < 16;
  extern __shared__ float4_t sd_red[];      // [wave][G][H][H][64 lanes]
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, j = lane & 15;
  int32_t t;
  if constexpr (SPLIT) {
    t = xcd_task(blockIdx.x, p.num_tasks);
  } else {
    t = xcd_task(blockIdx.x, (p.num_tasks + 3) / 4) * 4 + wave;
    if (t >= p.num_tasks) return;
  }
  const int32_t r = sload(p.tasks, 2 * (int64_t)t), q0 = sload(p.tasks, 2 * (int64_t)t + 1);
  const int32_t q_end = min(sload(p.row_ptr, r + 1), q0 + G * BG);
  __amdgpu_buffer_rsrc_t dyr = __builtin_amdgcn_make_buffer_rsrc((void*)p.dY, (short)0, (int)p.dy_bytes, 0x00020000);
  __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)p.X, (short)0, (int)p.x_bytes, 0x00020000);
  // c[e]: block column of group e (b >= 16: wave-uniform; b < 16: of this
  // lane's block j / b in the group); -1 past the task's last block
  int32_t c[G];
#pragma unroll
  for (int e = 0; e < G; ++e) {
    if constexpr (kSmall) {
      const int32_t q = q0 + e * BG + j / B;
      c[e] = q < q_end ? p.col_idx[q] : -1;
    } else {
      c[e] = q0 + e < q_end ? sload(p.col_idx, q0 + e) : -1;
    }
  }
  float4_t acc[G][H][H];
#pragma unroll
  for (int e = 0; e < G; ++e)
#pragma unroll
    for (int a = 0; a < H; ++a)
#pragma unroll
      for (int bb = 0; bb < H; ++bb) acc[e][a][bb] = float4_t{0.f, 0.f, 0.f, 0.f};
  // A step covers 64 values of n as two MFMAs: lane (g, .) takes the 16
  // consecutive values 64s + 16g .. +16, the first 8 in MFMA 0 and the next 8
  // in MFMA 1 (the same k order in A and B), so the four lanes of a row read
  // one whole 128-byte line per step.
  const int32_t steps = (p.n + 63) / 64, per = SPLIT ? (steps + 3) / 4 : steps;
  const int32_t s_lo = SPLIT ? min(steps, wave * per) : 0, s_hi = min(steps, s_lo + per);
  // rows of dY and X this lane loads (past the matrix: zero)
  const int64_t dy_row0 = kSmall ? (j < B ? (int64_t)r * B + j : (int64_t)p.m) : (int64_t)r * B + j;
  auto x_row = [&](int e, int bb) -> int64_t {
    if constexpr (kSmall) return c[e] >= 0 ? (int64_t)c[e] * B + (j % B) : (int64_t)p.k;
    else return (int64_t)c[e] * B + 16 * bb + j;
  };
  auto load = [&](int32_t s, u32x4 (&av)[2][H], u32x4 (&bv)[2][G][H]) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int32_t c0 = 64 * s + 16 * g + 8 * t;
#pragma unroll
      for (int a = 0; a < H; ++a) av[t][a] = load8(dyr, dy_row0 + 16 * a, p.m, p.lddy, c0, p.n);
#pragma unroll
      for (int e = 0; e < G; ++e)
#pragma unroll
        for (int bb = 0; bb < H; ++bb) {
          if constexpr (kSmall) bv[t][e][bb] = load8(xr, x_row(e, bb), p.k, p.ldx, c0, p.n);
          else bv[t][e][bb] = c[e] >= 0 ? load8(xr, x_row(e, bb), p.k, p.ldx, c0, p.n) : u32x4{0, 0, 0, 0};
        }
    }
  };
  auto mma = [&](const u32x4 (&av)[2][H], const u32x4 (&bv)[2][G][H]) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int e = 0; e < G; ++e) {
        if (q0 + e * BG >= q_end) continue;
#pragma unroll
        for (int bb = 0; bb < H; ++bb)
#pragma unroll
          for (int a = 0; a < H; ++a) acc[e][a][bb] = Mfma<T>::k32(av[t][a], bv[t][e][bb], acc[e][a][bb]);
      }
  };
  if (s_lo < s_hi) {
    u32x4 av[2][H], bv[2][G][H];
    load(s_lo, av, bv);
    for (int32_t s = s_lo; s < s_hi; ++s) {
      u32x4 an[2][H], bn[2][G][H];
      const bool more = s + 1 < s_hi;
      if (more) load(s + 1, an, bn);
      mma(av, bv);
      if (more) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
#pragma unroll
          for (int a = 0; a < H; ++a) av[t][a] = an[t][a];
#pragma unroll
          for (int e = 0; e < G; ++e)
#pragma unroll
            for (int bb = 0; bb < H; ++bb) bv[t][e][bb] = bn[t][e][bb];
        }
      }
    }
  }
  // D[4g + i][j] of tile (a, bb) of group e: b >= 16, element (16a + 4g + i,
  // 16bb + j) of block e; b < 16, element (4g + i, j % b) of block
  // e * 16 / b + j / b, for rows 4g + i < b only
  auto store = [&](int e, int a, int bb, const float4_t& v) {
    if constexpr (kSmall) {
      const int32_t q = q0 + e * BG + j / B;
      if (q >= q_end || 4 * g >= B) return;
      float* out = p.G + (int64_t)q * B * B;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (4 * g + i < B) out[(4 * g + i) * B + (j % B)] = v[i];
    } else {
      if (q0 + e >= q_end) return;
      float* out = p.G + (int64_t)(q0 + e) * B * B;
#pragma unroll
      for (int i = 0; i < 4; ++i) out[(16 * a + 4 * g + i) * B + 16 * bb + j] = v[i];
    }
  };
  if constexpr (!SPLIT) {
#pragma unroll
    for (int e = 0; e < G; ++e)
#pragma unroll
      for (int a = 0; a < H; ++a)
#pragma unroll
        for (int bb = 0; bb < H; ++bb) store(e, a, bb, acc[e][a][bb]);
    return;
  }
#pragma unroll
  for (int e = 0; e < G; ++e)
#pragma unroll
    for (int a = 0; a < H; ++a)
#pragma unroll
      for (int bb = 0; bb < H; ++bb) sd_red[(((wave * G + e) * H + a) * H + bb) * 64 + lane] = acc[e][a][bb];
  __syncthreads();
  // wave w finishes groups w, w + 4, ...
  for (int e = wave; e < G; e += 4) {
#pragma unroll
    for (int a = 0; a < H; ++a)
#pragma unroll
      for (int bb = 0; bb < H; ++bb) {
        float4_t v = sd_red[(((0 * G + e) * H + a) * H + bb) * 64 + lane];
#pragma unroll
        for (int w = 1; w < 4; ++w) v += sd_red[(((w * G + e) * H + a) * H + bb) * 64 + lane];
        store(e, a, bb, v);
      }
  }
}

// ------------------------------------------------------------------ tiled form
// For b = 16 and 32: a task is up to 64 MFMA tiles (16 x 16) of the nonzero
// blocks of one tile of kTile rows of dY by kTile rows of X (kTile / b block
// rows by kTile / b block columns). The workgroup walks n in chunks of kNK:
// each thread brings one dY row and one X row of the chunk into LDS (two
// buffers: the next chunk's loads are in flight while the current one is
// multiplied), and each wave multiplies its blocks' fragments out of LDS.
// Every dY and X row of the tile is read from memory once per task instead of
// once per block, which pays where a tile holds many blocks.
constexpr int kTile = 256;                 // rows of dY and of X per tile (one per thread)
constexpr int kNK = 32;                    // n values per chunk: one K = 32 MFMA step
constexpr int kLdw = kNK + 8;              // LDS row stride in elements (16-byte aligned, spreads banks)
constexpr int kTileMfmas = 16;             // MFMA tiles per wave
constexpr int kTiledLds = 2 * 2 * kTile * kLdw * 2;  // two buffers of dY and X rows: 80 KiB

struct TiledParams {
  const int32_t* tasks;  // [num_tasks][4]: tile row, tile column, first entry, count
  const int32_t* ent;    // [nnz][2]: CSR index, (block row in tile << 16) | block column in tile
  int32_t num_tasks;
  const void* dY;
  const void* X;
  float* G;
  int64_t lddy, ldx;
  int32_t m, k, n;
  uint32_t dy_bytes, x_bytes;
};

__device__ __forceinline__ void sync_lds() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0) only: the next chunk's global loads stay in flight
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// The chunk's loads: 512 rows (the tile's 256 dY rows, then its 256 X rows)
// of 32 values, four 16-byte segments per row; thread t takes segment t % 4
// of rows t / 4 + 64 i (i = 0 .. 7), so four consecutive lanes read one row's
// 64 contiguous bytes. Zero past m or k (buffer bounds) and past n (masked).
__device__ __forceinline__ void load_chunk(__amdgpu_buffer_rsrc_t dyr, __amdgpu_buffer_rsrc_t xr, const TiledParams& p,
                                           int64_t dy0, int64_t x0, int32_t c0, int tid, u32x4 (&v)[8]) {
  const int seg = tid & 3, r0 = tid >> 2;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int row = r0 + 64 * i;  // 0 .. 511
    if (i < 4) v[i] = load8(dyr, dy0 + row, p.m, p.lddy, c0 + 8 * seg, p.n);
    else v[i] = load8(xr, x0 + (row - kTile), p.k, p.ldx, c0 + 8 * seg, p.n);
  }
}

template <typename T, int B>
__global__ __launch_bounds__(256) void k_sddmm_tiled(TiledParams p) {
  constexpr int H = B / 16;
  constexpr int BW = kTileMfmas / (H * H);  // blocks per wave
  extern __shared__ uint4 tl_lds[];
  uint16_t* lds = (uint16_t*)tl_lds;  // [buf][dY, X][kTile][kLdw]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, j = lane & 15;
  const int32_t t = xcd_task(blockIdx.x, p.num_tasks);
  const int32_t tr = sload(p.tasks, 4 * (int64_t)t), tc = sload(p.tasks, 4 * (int64_t)t + 1);
  const int32_t first = sload(p.tasks, 4 * (int64_t)t + 2), count = sload(p.tasks, 4 * (int64_t)t + 3);
  // this wave's blocks: entries first + wave * BW .. (fewer in the last wave)
  const int32_t w0 = wave * BW, nb = max(0, min(BW, count - w0));
  int32_t q[BW], rl[BW], cl[BW];
#pragma unroll
  for (int e = 0; e < BW; ++e) {
    const bool on = e < nb;
    q[e] = on ? sload(p.ent, 2 * (int64_t)(first + w0 + e)) : 0;
    const int32_t rc = on ? sload(p.ent, 2 * (int64_t)(first + w0 + e) + 1) : 0;
    rl[e] = rc >> 16;
    cl[e] = rc & 0xFFFF;
  }
  __amdgpu_buffer_rsrc_t dyr = __builtin_amdgcn_make_buffer_rsrc((void*)p.dY, (short)0, (int)p.dy_bytes, 0x00020000);
  __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc((void*)p.X, (short)0, (int)p.x_bytes, 0x00020000);
  const int64_t dy0 = (int64_t)tr * kTile, x0 = (int64_t)tc * kTile;
  float4_t acc[BW][H][H];
#pragma unroll
  for (int e = 0; e < BW; ++e)
#pragma unroll
    for (int a = 0; a < H; ++a)
#pragma unroll
      for (int bb = 0; bb < H; ++bb) acc[e][a][bb] = float4_t{0.f, 0.f, 0.f, 0.f};
  auto stage = [&](int buf, const u32x4 (&v)[8]) {
    const int seg = tid & 3, r0 = tid >> 2;
#pragma unroll
    for (int i = 0; i < 8; ++i) *(u32x4*)(lds + (buf * 2 * kTile + r0 + 64 * i) * kLdw + 8 * seg) = v[i];
  };
  const int32_t chunks = (p.n + kNK - 1) / kNK;
  u32x4 v[8];
  load_chunk(dyr, xr, p, dy0, x0, 0, tid, v);
  stage(0, v);
  if (chunks > 1) load_chunk(dyr, xr, p, dy0, x0, kNK, tid, v);
  sync_lds();
  for (int32_t ch = 0; ch < chunks; ++ch) {
    const int buf = ch & 1;
    const uint16_t* ly = lds + (buf * 2 + 0) * kTile * kLdw;
    const uint16_t* lx = lds + (buf * 2 + 1) * kTile * kLdw;
    // a task lists its blocks by row, so consecutive blocks of a wave often
    // share their dY fragments: loaded once per run of one row
    u32x4 av[H];
#pragma unroll
    for (int e = 0; e < BW; ++e) {
      if (e < nb) {
        if (e == 0 || rl[e] != rl[e - 1]) {
#pragma unroll
          for (int a = 0; a < H; ++a) av[a] = *(const u32x4*)(ly + (rl[e] * B + 16 * a + j) * kLdw + 8 * g);
        }
#pragma unroll
        for (int bb = 0; bb < H; ++bb) {
          const u32x4 bv = *(const u32x4*)(lx + (cl[e] * B + 16 * bb + j) * kLdw + 8 * g);
#pragma unroll
          for (int a = 0; a < H; ++a) acc[e][a][bb] = Mfma<T>::k32(av[a], bv, acc[e][a][bb]);
        }
      }
    }
    if (ch + 1 < chunks) {
      stage(buf ^ 1, v);  // chunk ch + 1 (its loads were issued one chunk ago)
      if (ch + 2 < chunks) load_chunk(dyr, xr, p, dy0, x0, (ch + 2) * kNK, tid, v);
    }
    sync_lds();  // chunk ch consumed by every wave; chunk ch + 1 staged
  }
  // D[4g + i][j] of tile (a, bb): element (16a + 4g + i, 16bb + j) of the block
#pragma unroll
  for (int e = 0; e < BW; ++e) {
    if (e < nb) {
      float* out = p.G + (int64_t)q[e] * B * B;
#pragma unroll
      for (int a = 0; a < H; ++a)
#pragma unroll
        for (int bb = 0; bb < H; ++bb)
#pragma unroll
          for (int i = 0; i < 4; ++i) out[(16 * a + 4 * g + i) * B + 16 * bb + j] = acc[e][a][bb][i];
    }
  }
}

template <typename T>
spmm_status_t launch_tiled_t(const TiledParams& p, int32_t b, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    SPMM_HIP(hipFuncSetAttribute((const void*)k_sddmm_tiled<T, 16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 kTiledLds));
    SPMM_HIP(hipFuncSetAttribute((const void*)k_sddmm_tiled<T, 32>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 kTiledLds));
    attr = true;
  }
  if (b == 16) hipLaunchKernelGGL((k_sddmm_tiled<T, 16>), dim3((unsigned)p.num_tasks), dim3(256), kTiledLds, s, p);
  else hipLaunchKernelGGL((k_sddmm_tiled<T, 32>), dim3((unsigned)p.num_tasks), dim3(256), kTiledLds, s, p);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

template <typename T>
spmm_status_t launch_t(const SddmmParams& p, int32_t b, hipStream_t s) {
  // Few tasks: split n over the 4 waves of a workgroup so the chip fills;
  // many tasks: one task per wave over all of n (no reduction in LDS).
  static const int cus = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 256;
    return v > 0 ? v : 256;
  }();
  if (p.num_tasks <= 32 * cus) {
    const unsigned grid = (unsigned)p.num_tasks;
    if (b == 1) hipLaunchKernelGGL((k_sddmm<T, 1, true>), dim3(grid), dim3(256), sddmm_lds_bytes<1>(), s, p);
    else if (b == 4) hipLaunchKernelGGL((k_sddmm<T, 4, true>), dim3(grid), dim3(256), sddmm_lds_bytes<4>(), s, p);
    else if (b == 8) hipLaunchKernelGGL((k_sddmm<T, 8, true>), dim3(grid), dim3(256), sddmm_lds_bytes<8>(), s, p);
    else if (b == 16) hipLaunchKernelGGL((k_sddmm<T, 16, true>), dim3(grid), dim3(256), sddmm_lds_bytes<16>(), s, p);
    else hipLaunchKernelGGL((k_sddmm<T, 32, true>), dim3(grid), dim3(256), sddmm_lds_bytes<32>(), s, p);
  } else {
    const unsigned grid = (unsigned)ceil_div(p.num_tasks, 4);
    if (b == 1) hipLaunchKernelGGL((k_sddmm<T, 1, false>), dim3(grid), dim3(256), 0, s, p);
    else if (b == 4) hipLaunchKernelGGL((k_sddmm<T, 4, false>), dim3(grid), dim3(256), 0, s, p);
    else if (b == 8) hipLaunchKernelGGL((k_sddmm<T, 8, false>), dim3(grid), dim3(256), 0, s, p);
    else if (b == 16) hipLaunchKernelGGL((k_sddmm<T, 16, false>), dim3(grid), dim3(256), 0, s, p);
    else hipLaunchKernelGGL((k_sddmm<T, 32, false>), dim3(grid), dim3(256), 0, s, p);
  }
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

}  // namespace

int32_t sddmm_tiled_tile_blocks(int32_t b) { return kTile / b; }
int32_t sddmm_tiled_task_blocks(int32_t b) { return 4 * kTileMfmas / ((b / 16) * (b / 16)); }

spmm_status_t launch_sddmm_tiled(spmm_dtype_t t, int32_t b, const int32_t* tasks, const int32_t* ent,
                                 int32_t num_tasks, int64_t m, int64_t k, int64_t n, const void* dY, int64_t lddy,
                                 const void* X, int64_t ldx, float* G, hipStream_t s) {
  if (b != 16 && b != 32) return fail(SPMM_ERR_UNSUPPORTED, "the tiled SDDMM handles block sizes 16 and 32");
  if (num_tasks == 0 || n == 0) return SPMM_OK;
  const int64_t dyb = m * lddy * 2, xb = k * ldx * 2;
  if (dyb >= (int64_t)INT32_MAX || xb >= (int64_t)INT32_MAX)
    return fail(SPMM_ERR_UNSUPPORTED, "dY or X larger than 2 GiB is not supported");
  TiledParams p;
  p.tasks = tasks;
  p.ent = ent;
  p.num_tasks = num_tasks;
  p.dY = dY;
  p.X = X;
  p.G = G;
  p.lddy = lddy;
  p.ldx = ldx;
  p.m = (int32_t)m;
  p.k = (int32_t)k;
  p.n = (int32_t)n;
  p.dy_bytes = (uint32_t)dyb;
  p.x_bytes = (uint32_t)xb;
  if (t == SPMM_F16) return launch_tiled_t<_Float16>(p, b, s);
  if (t == SPMM_BF16) return launch_tiled_t<__bf16>(p, b, s);
  return fail(SPMM_ERR_UNSUPPORTED, "SDDMM needs FP16 or BF16 dY and X");
}

int32_t sddmm_task_blocks(int32_t b) {
  switch (b) {
    case 1: return task_blocks<1>();
    case 4: return task_blocks<4>();
    case 8: return task_blocks<8>();
    case 16: return task_blocks<16>();
    default: return task_blocks<32>();
  }
}

spmm_status_t launch_sddmm(spmm_dtype_t t, int32_t b, const int32_t* row_ptr, const int32_t* col_idx,
                           const int32_t* tasks, int32_t num_tasks, int64_t m, int64_t k, int64_t n, const void* dY,
                           int64_t lddy, const void* X, int64_t ldx, float* G, hipStream_t s) {
  if (b != 1 && b != 4 && b != 8 && b != 16 && b != 32)
    return fail(SPMM_ERR_UNSUPPORTED, "SDDMM handles block sizes 1, 4, 8, 16 and 32");
  if (num_tasks == 0 || n == 0) return SPMM_OK;
  const int64_t dyb = m * lddy * 2, xb = k * ldx * 2;
  if (dyb >= (int64_t)INT32_MAX || xb >= (int64_t)INT32_MAX)
    return fail(SPMM_ERR_UNSUPPORTED, "dY or X larger than 2 GiB is not supported");
  SddmmParams p;
  p.row_ptr = row_ptr;
  p.col_idx = col_idx;
  p.tasks = tasks;
  p.num_tasks = num_tasks;
  p.dY = dY;
  p.X = X;
  p.G = G;
  p.lddy = lddy;
  p.ldx = ldx;
  p.m = (int32_t)m;
  p.k = (int32_t)k;
  p.n = (int32_t)n;
  p.dy_bytes = (uint32_t)dyb;
  p.x_bytes = (uint32_t)xb;
  if (t == SPMM_F16) return launch_t<_Float16>(p, b, s);
  if (t == SPMM_BF16) return launch_t<__bf16>(p, b, s);
  return fail(SPMM_ERR_UNSUPPORTED, "SDDMM needs FP16 or BF16 dY and X");
}

}  // namespace spmm
