// One-launch dynamic call (Section 3.3, Appendix A.2: the pattern arrives
// with the call and is re-bucketed on the device), for b = 16 with W in the X
// type (FP16 or BF16).
//
// The encoder and the product share one launch: a workgroup of 16 waves owns
// block row r and a group of four column tiles, reads the whole COO list of
// the call in one round of loads, validates it (so every workgroup reaches
// the same status, and on an error all of them skip the product and leave Y
// alone), counts the entries of the rows above r (its row's first CSR
// position) and keeps its own row's entries in LDS as keys (column << 16 |
// input index). Sorted, the keys are the row's CSR order, the canonical
// (column, input index) order of every other encoder; the workgroup of the
// first tile group writes that block-CSR (for an export). Then four waves per
// column tile run the split-row product on the keys: the w-th wave of a tile
// takes the w-th pair-aligned quarter of the row, and the partial sums are
// added in wave order. That is the every-row split form of the row kernel, so
// the result equals a two-launch call (or a static plan) that runs that form,
// bit for bit. No workgroup waits for another.
#include "spmm_row.h"

namespace spmm {
namespace {

using namespace row;

constexpr int kFusedThreads = 1024;
constexpr int kFusedU = 8;       // entries per thread loaded together while scanning (8192 a round)
constexpr int kTilesPerGroup = 4;  // column tiles of a workgroup, four waves each

struct FusedParams {
  RowProblem pr;  // W: the call's values in input order; Y, X as for the row kernel
  const int32_t* nnz_dev;
  const int32_t* rows;
  const int32_t* cols;
  int32_t max_nnz, kb;
  int32_t num_units;  // mb x column-tile groups
  int32_t* row_ptr;   // the call's block-CSR, for an export
  int32_t* col_idx;
  int32_t* src;
  int32_t* status;
  int32_t* status_out;
  int32_t* nnz_last;
};

// Sorts keys[0, n) ascending in LDS (distinct keys: the input index is part of
// each). Up to 64 in one wave by rank (a key's place is the number of smaller
// keys, counted over the wave's lanes), up to 8 per thread by rank over LDS,
// longer lists by a bitonic network over the next power of two (the padding
// keys, all ones, sort last; the caller sized the array for them).
__device__ __forceinline__ void sort_keys(uint32_t* keys, int32_t n, int tid) {
  if (n <= 64) {
    if (tid < 64) {
      const uint32_t mine = tid < n ? keys[tid] : 0xffffffffu;
      int32_t rank = 0;
      for (int32_t j = 0; j < n; ++j) rank += (uint32_t)__builtin_amdgcn_readlane((int)mine, j) < mine ? 1 : 0;
      if (tid < n) keys[rank] = mine;  // the wave read every key before any lane writes
    }
    __syncthreads();
    return;
  }
  if (n <= 8 * kFusedThreads) {
    uint32_t mine[8];
    int32_t rank[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int32_t i = tid + u * kFusedThreads;
      mine[u] = i < n ? keys[i] : 0u;
      rank[u] = 0;
    }
    for (int32_t j = 0; j < n; ++j) {
      const uint32_t kj = keys[j];
#pragma unroll
      for (int u = 0; u < 8; ++u) rank[u] += kj < mine[u] ? 1 : 0;
    }
    __syncthreads();  // every key read before any is moved
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (tid + u * kFusedThreads < n) keys[rank[u]] = mine[u];
    __syncthreads();
    return;
  }
  int32_t P = 1;
  while (P < n) P <<= 1;
  for (int32_t i = n + tid; i < P; i += kFusedThreads) keys[i] = 0xffffffffu;
  __syncthreads();
  for (int32_t size = 2; size <= P; size <<= 1) {
    for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (int32_t i = tid; i < P / 2; i += kFusedThreads) {
        const int32_t lo = 2 * i - (i & (stride - 1)), hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint32_t a = keys[lo], b = keys[hi];
        if ((a > b) == up) {
          keys[lo] = b;
          keys[hi] = a;
        }
      }
      __syncthreads();
    }
  }
}

template <typename XT, typename YT, int NS>
__global__ __launch_bounds__(kFusedThreads) void k_dyn_fused(FusedParams f) {
  extern __shared__ uint32_t fz_keys[];  // [sort capacity] keys; then the waves' partial sums
  __shared__ int32_t flag[3];            // [0] error, [1] kept entries, [2] nnz
  __shared__ int32_t wsum[kFusedThreads / 64];
  const RowProblem& p = f.pr;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int32_t unit = xcd_unit(blockIdx.x, f.num_units);  // an XCD's units share column tiles
  const int32_t r = unit % p.mb, tg = unit / p.mb;
  if (tid == 0) {
    const int32_t nnz = *f.nnz_dev;
    flag[0] = (nnz < 0 || nnz > f.max_nnz) ? (int32_t)SPMM_ERR_CAPACITY : 0;
    flag[1] = 0;
    flag[2] = nnz;
  }
  __syncthreads();
  const int32_t nnz = flag[2];
  int32_t above = 0;  // entries of rows before r seen by this thread
  if (flag[0] == 0) {
    for (int32_t base = 0; base < nnz; base += kFusedThreads * kFusedU) {
      int32_t er[kFusedU], ec[kFusedU];
#pragma unroll
      for (int u = 0; u < kFusedU; ++u) {
        const int32_t e = base + u * kFusedThreads + tid;
        er[u] = e < nnz ? f.rows[e] : 0;
        ec[u] = e < nnz ? f.cols[e] : 0;
      }
#pragma unroll
      for (int u = 0; u < kFusedU; ++u) {
        const int32_t e = base + u * kFusedThreads + tid;
        if (e >= nnz) continue;
        const int32_t er_ = er[u], ec_ = ec[u];
        if (er_ < 0 || er_ >= p.mb || ec_ < 0 || ec_ >= f.kb) {
          atomicMax(&flag[0], (int32_t)SPMM_ERR_BAD_INDEX);
          continue;
        }
        if (er_ < r) {
          ++above;
        } else if (er_ == r) {
          const int32_t slot = atomicAdd(&flag[1], 1);
          fz_keys[slot] = ((uint32_t)ec_ << 16) | (uint32_t)e;
        }
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) above += __shfl_xor(above, off);
  if (lane == 0) wsum[wave] = above;
  __syncthreads();
  const int32_t err = flag[0];
  if (err) {  // every workgroup read the same entries: the same status
    if (blockIdx.x == 0 && tid == 0) {
      *f.status = err;
      if (f.status_out) *f.status_out = err;
    }
    return;
  }
  int32_t first = 0;
#pragma unroll
  for (int w = 0; w < kFusedThreads / 64; ++w) first += wsum[w];
  const int32_t kept = flag[1];
  sort_keys(fz_keys, kept, tid);
  if (tg == 0) {  // the row's block-CSR and, once, the call's status
    for (int32_t i = tid; i < kept; i += kFusedThreads) {
      const uint32_t key = fz_keys[i];
      f.col_idx[first + i] = (int32_t)(key >> 16);
      f.src[first + i] = (int32_t)(key & 0xffffu);
    }
    if (tid == 0) {
      f.row_ptr[r] = first;
      if (r == p.mb - 1) f.row_ptr[p.mb] = first + kept;
      if (r == 0) {
        *f.status = 0;
        if (f.status_out) *f.status_out = 0;
        if (f.nnz_last) *f.nnz_last = nnz;
      }
    }
  }
  // the split-row product on the sorted keys: quarter qw of tile tl
  const int tl = wave >> 2, qw = wave & 3;
  const int32_t t = tg * kTilesPerGroup + tl;
  const bool live = t * (16 * NS) < p.n;
  const int32_t n0 = t * (16 * NS);
  const int32_t seg = ((kept + 7) / 8) * 2;  // a quarter of the row, rounded up to whole pairs
  const int32_t qa = min(kept, qw * seg), qb = live ? min(kept, qa + seg) : qa;
  float4_t acc[1][NS];
  row_acc<XT, XT, 16, NS, LdsKeys>(p, qa, qb, n0, lane, acc, LdsKeys{fz_keys});
  __syncthreads();  // every wave is done with the keys: their LDS takes the partial sums
  float4_t* red = (float4_t*)fz_keys + (int64_t)tl * 3 * NS * 64;
  if (qw > 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) red[((qw - 1) * NS + s) * 64 + lane] = acc[0][s];
  }
  __syncthreads();
  if (qw == 0 && live) {
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
      for (int s = 0; s < NS; ++s) acc[0][s] += red[(w * NS + s) * 64 + lane];
    row_store<YT, 16, NS>(p, r, n0, lane, acc);
  }
}

// LDS of a launch: the keys of a row (at most max_nnz, padded to a power of
// two for the bitonic sort when more than 8 per thread) or the partial sums of
// three waves per tile, whichever is larger.
size_t fused_lds_bytes(int32_t max_nnz, int ns) {
  int64_t cap = max_nnz;
  if (cap > 8 * kFusedThreads) {
    int64_t P = 1;
    while (P < cap) P <<= 1;
    cap = P;
  }
  return std::max<size_t>(sizeof(uint32_t) * (size_t)cap, (size_t)kTilesPerGroup * split_lds_bytes(16, ns));
}

constexpr size_t kFusedLdsMax = 128 * 1024;

template <typename XT, typename YT, int NS>
spmm_status_t launch_fused_ns(const FusedParams& f, size_t lds, unsigned grid, hipStream_t s) {
  static bool attr_set = false;  // dynamic LDS beyond 64 KiB must be allowed per kernel
  if (!attr_set) {
    SPMM_HIP(hipFuncSetAttribute((const void*)k_dyn_fused<XT, YT, NS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)kFusedLdsMax));
    attr_set = true;
  }
  hipLaunchKernelGGL((k_dyn_fused<XT, YT, NS>), dim3(grid), dim3(kFusedThreads), lds, s, f);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

template <typename XT, typename YT>
spmm_status_t launch_fused_t(const FusedParams& f, int ns, size_t lds, unsigned grid, hipStream_t s) {
  if (ns == 8) return launch_fused_ns<XT, YT, 8>(f, lds, grid, s);
  if (ns == 4) return launch_fused_ns<XT, YT, 4>(f, lds, grid, s);
  if (ns == 2) return launch_fused_ns<XT, YT, 2>(f, lds, grid, s);
  return fail(SPMM_ERR_INVALID_ARG, "column tile variant must be 2, 4 or 8");
}

}  // namespace

bool dynamic_fused_eligible(int32_t b, spmm_dtype_t w, spmm_dtype_t x, spmm_dtype_t y, int64_t k, int32_t mb,
                            int32_t kb, int64_t max_nnz) {
  if (b != 16 || w != x || (x != SPMM_F16 && x != SPMM_BF16) || (y != x && y != SPMM_F32)) return false;
  if (k % 16 != 0 || mb < 1 || kb > 65536 || max_nnz < 1 || max_nnz > 65536) return false;
  return fused_lds_bytes((int32_t)max_nnz, 8) <= kFusedLdsMax;
}

// The rule's tile width for the one-launch form: 4 column tiles of 16 per
// wave (2 for n <= 32): a block row's four tiles then cover 256 columns.
int32_t dynamic_fused_ns(int64_t n) { return n > 32 ? 4 : 2; }

// The rule: one launch where the grid fills no more than one round of the
// chip (one 16-wave workgroup per CU) and the redundant scans stay small, at
// most 2^22 entries read over the grid. At m = k = 4096 with 8192 blocks at
// most, that is n <= 256, where one launch measured 14 - 16 us per call
// against 17 us for the encoder and the every-row split form; at n = 512 the
// two launches are faster (19.4 against 20.9 us).
bool dynamic_fused_preferred(int32_t mb, int64_t n, int64_t max_nnz) {
  if (const char* e = getenv("SPMM_DYN_FUSED")) return e[0] == '1';
  const int64_t units = (int64_t)mb * ceil_div(n, 16 * dynamic_fused_ns(n) * kTilesPerGroup);
  return max_nnz * units <= ((int64_t)1 << 22) && units <= device_cu_count();
}

spmm_status_t launch_dynamic_fused(const RunArgs& a, const int32_t* nnz_dev, const int32_t* rows, const int32_t* cols,
                                   int32_t max_nnz, int32_t kb, int32_t* row_ptr, int32_t* col_idx, int32_t* src,
                                   int32_t* status, int32_t* status_out, int32_t* nnz_last, hipStream_t s) {
  if (!dynamic_fused_eligible(a.plan.b, a.wt, a.xt, a.yt, a.plan.k, a.plan.mb, kb, max_nnz))
    return fail(SPMM_ERR_UNSUPPORTED, "the one-launch dynamic call needs b = 16, W in the X type and a small capacity");
  if ((int64_t)a.plan.k * a.ldx * 2 >= (int64_t)INT32_MAX)
    return fail(SPMM_ERR_UNSUPPORTED, "X larger than 2 GiB is not supported");
  if (a.n < 1) return fail(SPMM_ERR_INVALID_ARG, "the one-launch call needs n >= 1");
  const int ns = a.ns;
  FusedParams f;
  RunArgs b = a;
  b.heavy_rows = nullptr;
  b.num_heavy = 0;
  b.light_rows = nullptr;
  b.part = nullptr;
  b.split_all = false;
  f.pr = row::row_problem(b, nullptr, nullptr);
  f.pr.w_index = nullptr;
  f.nnz_dev = nnz_dev;
  f.rows = rows;
  f.cols = cols;
  f.max_nnz = max_nnz;
  f.kb = kb;
  const int64_t units = (int64_t)a.plan.mb * ceil_div(a.n, 16 * ns * kTilesPerGroup);
  if (units > (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "too many work units");
  f.num_units = (int32_t)units;
  f.row_ptr = row_ptr;
  f.col_idx = col_idx;
  f.src = src;
  f.status = status;
  f.status_out = status_out;
  f.nnz_last = nnz_last;
  const size_t lds = fused_lds_bytes(max_nnz, ns);
  if (a.xt == SPMM_F16)
    return a.yt == SPMM_F32 ? launch_fused_t<_Float16, float>(f, ns, lds, (unsigned)units, s)
                            : launch_fused_t<_Float16, _Float16>(f, ns, lds, (unsigned)units, s);
  return a.yt == SPMM_F32 ? launch_fused_t<__bf16, float>(f, ns, lds, (unsigned)units, s)
                          : launch_fused_t<__bf16, __bf16>(f, ns, lds, (unsigned)units, s);
}

}  // namespace spmm
