// Dynamic-mode re-bucketing straight into block-CSR (PopSparse Section 3.3 and
// Appendix A.2: the pattern arrives with every run and is distributed into
// buckets sized from the declared maximum). Here a bucket is a block row:
//   1. validate indices and count entries per block row (integer atomics);
//   2. exclusive scan of the counts -> row_ptr (one workgroup);
//   3. scatter every entry into its row (slots handed out by atomics);
//   4. sort each row by (block column, input index): the result no longer
//      depends on the order the atomics handed out slots;
//   5. gather the values (and FP8 scales) into block-CSR order, zeroing the
//      part of edge blocks beyond column k;
// plus the cost-balanced panels of the row groups. Every kernel reads the
// entry count from device memory and stops when the status word is set.
#include <algorithm>
#include <cstdlib>

#include "common.h"

namespace spmm {
namespace {

__global__ void k_dyn_zero(int32_t* __restrict__ a, int64_t na, int32_t* __restrict__ status) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *status = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < na; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0;
}

__global__ void k_dyn_row_count(const int32_t* __restrict__ nnz_dev, int32_t max_nnz, const int32_t* __restrict__ rows,
                                const int32_t* __restrict__ cols, int32_t mb, int32_t kb, int32_t* __restrict__ row_cnt,
                                int32_t* __restrict__ status) {
  const int32_t nnz = *nnz_dev;
  if (nnz < 0 || nnz > max_nnz) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicMax(status, (int32_t)SPMM_ERR_CAPACITY);
    return;
  }
  for (int32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += gridDim.x * blockDim.x) {
    const int32_t r = rows[e], c = cols[e];
    if (r < 0 || r >= mb || c < 0 || c >= kb) {
      atomicMax(status, (int32_t)SPMM_ERR_BAD_INDEX);
      continue;
    }
    atomicAdd(&row_cnt[r], 1);
  }
}

// One workgroup of 1024 threads: exclusive scan of mb counts into row_ptr[0..mb].
__global__ __launch_bounds__(1024) void k_dyn_scan_rows(const int32_t* __restrict__ cnt, int32_t mb,
                                                        int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ status) {
  if (*status) return;
  __shared__ int32_t sh[1024];
  const int tid = threadIdx.x;
  const int per = (mb + 1023) / 1024;
  const int lo = min(mb, tid * per), hi = min(mb, lo + per);
  int32_t s = 0;
  for (int i = lo; i < hi; ++i) s += cnt[i];
  sh[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int32_t add = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += add;
    __syncthreads();
  }
  int32_t run = sh[tid] - s;
  for (int i = lo; i < hi; ++i) {
    row_ptr[i] = run;
    run += cnt[i];
  }
  if (tid == 1023) row_ptr[mb] = sh[1023];
}

__global__ void k_dyn_row_scatter(const int32_t* __restrict__ nnz_dev, const int32_t* __restrict__ rows,
                                  const int32_t* __restrict__ cols, const int32_t* __restrict__ row_ptr,
                                  int32_t* __restrict__ fill, int32_t* __restrict__ col_idx, int32_t* __restrict__ src,
                                  const int32_t* __restrict__ status) {
  if (*status) return;
  const int32_t nnz = *nnz_dev;
  for (int32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += gridDim.x * blockDim.x) {
    const int32_t r = rows[e];
    const int32_t pos = row_ptr[r] + atomicAdd(&fill[r], 1);
    col_idx[pos] = cols[e];
    src[pos] = e;
  }
}

// ------------------------------------------------------------------ histogram encode
// The multi-kernel encode without global atomics (a counting sort by block
// row): workgroup w takes entries [w chunk, (w + 1) chunk) and counts them per
// block row in LDS; a scan over the workgroups, per block row, turns the
// counts into each workgroup's first slot within the row and the row totals;
// the row totals are scanned into row_ptr; each workgroup then places its
// entries from its own slots with LDS atomics. The order inside a row is
// canonicalised by k_dyn_row_sort afterwards.
constexpr int kHistU = 8;        // entries per thread loaded together
constexpr int kHistChunk = 4096; // entries per workgroup (at most 256 workgroups)

__global__ __launch_bounds__(256) void k_dyn_hist(const int32_t* __restrict__ nnz_dev, int32_t max_nnz,
                                                  const int32_t* __restrict__ rows, const int32_t* __restrict__ cols,
                                                  int32_t mb, int32_t kb, int32_t chunk, int32_t* __restrict__ hist,
                                                  int32_t* __restrict__ status) {
  extern __shared__ int32_t hcnt[];  // [mb]
  const int32_t nnz = *nnz_dev;
  if (nnz < 0 || nnz > max_nnz) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicMax(status, (int32_t)SPMM_ERR_CAPACITY);
    return;
  }
  const int tid = threadIdx.x;
  for (int32_t r = tid; r < mb; r += 256) hcnt[r] = 0;
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min((int64_t)nnz, lo + chunk);
  for (int64_t base = lo; base < hi; base += 256 * kHistU) {
    int32_t er[kHistU], ec[kHistU];
#pragma unroll
    for (int u = 0; u < kHistU; ++u) {
      const int64_t e = base + u * 256 + tid;
      er[u] = e < hi ? rows[e] : 0;
      ec[u] = e < hi ? cols[e] : 0;
    }
#pragma unroll
    for (int u = 0; u < kHistU; ++u) {
      if (base + u * 256 + tid >= hi) continue;
      if (er[u] < 0 || er[u] >= mb || ec[u] < 0 || ec[u] >= kb) {
        atomicMax(status, (int32_t)SPMM_ERR_BAD_INDEX);
        continue;
      }
      atomicAdd(&hcnt[er[u]], 1);
    }
  }
  __syncthreads();
  for (int32_t r = tid; r < mb; r += 256) hist[(int64_t)blockIdx.x * mb + r] = hcnt[r];
}

// One thread per block row: hist[w][r] becomes the entries of row r in the
// workgroups before w; row_cnt[r] the row's total.
__global__ void k_dyn_hist_scan(int32_t* __restrict__ hist, int32_t wgs, int32_t mb, int32_t* __restrict__ row_cnt,
                                const int32_t* __restrict__ status) {
  if (*status) return;
  const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= mb) return;
  int32_t run = 0;
  int32_t w = 0;
  for (; w + 8 <= wgs; w += 8) {
    int32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = hist[(int64_t)(w + u) * mb + r];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      hist[(int64_t)(w + u) * mb + r] = run;
      run += v[u];
    }
  }
  for (; w < wgs; ++w) {
    const int32_t v = hist[(int64_t)w * mb + r];
    hist[(int64_t)w * mb + r] = run;
    run += v;
  }
  row_cnt[r] = run;
}

__global__ __launch_bounds__(256) void k_dyn_hist_scatter(const int32_t* __restrict__ nnz_dev,
                                                          const int32_t* __restrict__ rows,
                                                          const int32_t* __restrict__ cols, int32_t mb, int32_t chunk,
                                                          const int32_t* __restrict__ hist,
                                                          const int32_t* __restrict__ row_ptr,
                                                          int32_t* __restrict__ col_idx, int32_t* __restrict__ src,
                                                          const int32_t* __restrict__ status) {
  if (*status) return;
  extern __shared__ int32_t slot[];  // [mb] next free position of each block row for this workgroup
  const int tid = threadIdx.x;
  for (int32_t r = tid; r < mb; r += 256) slot[r] = row_ptr[r] + hist[(int64_t)blockIdx.x * mb + r];
  __syncthreads();
  const int32_t nnz = *nnz_dev;
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min((int64_t)nnz, lo + chunk);
  for (int64_t base = lo; base < hi; base += 256 * kHistU) {
    int32_t er[kHistU], ec[kHistU];
#pragma unroll
    for (int u = 0; u < kHistU; ++u) {
      const int64_t e = base + u * 256 + tid;
      er[u] = e < hi ? rows[e] : 0;
      ec[u] = e < hi ? cols[e] : 0;
    }
#pragma unroll
    for (int u = 0; u < kHistU; ++u) {
      const int64_t e = base + u * 256 + tid;
      if (e >= hi) continue;
      const int32_t pos = atomicAdd(&slot[er[u]], 1);
      col_idx[pos] = ec[u];
      src[pos] = (int32_t)e;
    }
  }
}

// One workgroup per block row orders the row's entries by (column, input
// index). Rows of at most kRowBmMax entries whose block columns all differ
// (the usual case) are placed through a column bitmap: each entry sets its
// column's bit (a repeated column is detected there), an exclusive scan of
// the words' bit counts gives each word the rank of its first entry, and an
// entry's rank is that plus the set bits below its column in its word. All
// of the row is read before any of it is written back in place. Other rows rank each entry against all others of the row, from LDS
// when the row fits, else from a global copy.
constexpr int kSortLds = 2048;
constexpr int kRowBmU = 8;                    // entries per thread
constexpr int kRowBmMax = 256 * kRowBmU;      // longest row placed through the bitmap
constexpr int kRowBmWords = 2048;             // bitmap words: block columns up to 65536
__global__ __launch_bounds__(256) void k_dyn_row_sort(const int32_t* __restrict__ row_ptr,
                                                      int32_t* __restrict__ col_idx, int32_t* __restrict__ src,
                                                      int32_t* __restrict__ tmp_col, int32_t* __restrict__ tmp_src,
                                                      int32_t kb, const int32_t* __restrict__ status) {
  if (*status) return;
  __shared__ int32_t sc[kSortLds], ss[kSortLds];
  __shared__ uint32_t bm[kRowBmWords];
  __shared__ int32_t wsum[4];
  __shared__ int32_t repeat;
  const int32_t r = blockIdx.x;
  const int32_t lo = row_ptr[r], hi = row_ptr[r + 1], len = hi - lo;
  if (len <= 1) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int32_t wpr = (kb + 31) >> 5;
  if (len <= kRowBmMax && wpr <= kRowBmWords) {
    for (int32_t i = tid; i < wpr; i += 256) bm[i] = 0;
    if (tid == 0) repeat = 0;
    __syncthreads();
    int32_t ec[kRowBmU], es[kRowBmU];
#pragma unroll
    for (int u = 0; u < kRowBmU; ++u) {
      const int32_t i = u * 256 + tid;
      ec[u] = i < len ? col_idx[lo + i] : 0;
      es[u] = i < len ? src[lo + i] : 0;
    }
    // every read of the row completes before the barrier (the columns feed the
    // bitmap, the sources are staged in LDS), so the in-place writes after it
    // cannot overtake a read
#pragma unroll
    for (int u = 0; u < kRowBmU; ++u) {
      if (u * 256 + tid >= len) continue;
      sc[u * 256 + tid] = es[u];
      const uint32_t bit = 1u << (ec[u] & 31);
      if (atomicOr(&bm[ec[u] >> 5], bit) & bit) repeat = 1;
    }
    __syncthreads();
    if (!repeat) {
      // exclusive scan of the words' bit counts: each thread a contiguous chunk
      int32_t* wpos = ss;  // [wpr] (ss is free on this path)
      const int32_t per = (wpr + 255) / 256;
      const int32_t a = min(wpr, tid * per), b = min(wpr, a + per);
      int32_t sum = 0;
      for (int32_t i = a; i < b; ++i) sum += __popc(bm[i]);
      int32_t incl = sum;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int32_t t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
      }
      if (lane == 63) wsum[wave] = incl;
      __syncthreads();
      int32_t run = incl - sum;
      for (int w = 0; w < wave; ++w) run += wsum[w];
      for (int32_t i = a; i < b; ++i) {
        wpos[i] = run;
        run += __popc(bm[i]);
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kRowBmU; ++u) {
        if (u * 256 + tid >= len) continue;
        const int32_t w = ec[u] >> 5;
        const int32_t pos = lo + wpos[w] + __popc(bm[w] & ((1u << (ec[u] & 31)) - 1u));
        col_idx[pos] = ec[u];
        src[pos] = sc[u * 256 + tid];
      }
      return;
    }
    // a repeated column: the pairwise ranking below (all threads read `repeat`
    // after the same barrier, so the whole workgroup takes it)
  }
  const bool in_lds = len <= kSortLds;
  for (int32_t i = threadIdx.x; i < len; i += blockDim.x) {
    const int32_t c = col_idx[lo + i], v = src[lo + i];
    if (in_lds) {
      sc[i] = c;
      ss[i] = v;
    } else {
      tmp_col[lo + i] = c;
      tmp_src[lo + i] = v;
    }
  }
  __syncthreads();
  for (int32_t i = threadIdx.x; i < len; i += blockDim.x) {
    const int32_t kc = in_lds ? sc[i] : tmp_col[lo + i], ks = in_lds ? ss[i] : tmp_src[lo + i];
    int32_t rank = 0;
    for (int32_t t = 0; t < len; ++t) {
      const int32_t c = in_lds ? sc[t] : tmp_col[lo + t], s2 = in_lds ? ss[t] : tmp_src[lo + t];
      rank += (c < kc) || (c == kc && s2 < ks);
    }
    col_idx[lo + rank] = kc;
    src[lo + rank] = ks;
  }
}

template <typename T>
__global__ void k_dyn_gather(const int32_t* __restrict__ nnz_dev, const int32_t* __restrict__ src,
                             const int32_t* __restrict__ col_idx, int32_t b, int32_t k, const T* __restrict__ vin,
                             T* __restrict__ vout, const float* __restrict__ sin, float* __restrict__ sout,
                             const int32_t* __restrict__ status) {
  if (*status) return;
  const int64_t nnz = *nnz_dev;
  const int64_t bb = (int64_t)b * b;
  const int32_t krem = k - (k / b) * b;
  const int32_t kb_last = (k + b - 1) / b - 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nnz * bb; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i / bb, w = i - e * bb;
    T v = vin[(int64_t)src[e] * bb + w];
    if (krem && col_idx[e] == kb_last && (int32_t)(w % b) >= krem) v = T(0);
    vout[i] = v;
    if (w == 0 && sin) sout[e] = sin[src[e]];
  }
}

// ------------------------------------------------------------------ one-workgroup builder
// The whole encode of one dynamic call in a single workgroup of 1024 threads,
// with the entries staged in LDS: validate and count per row (LDS atomics),
// exclusive scan, scatter into LDS, rank each row's entries by (column, input
// index) and write them to block-CSR in place, group costs, their prefix and
// the panel boundaries, then the status words. Used when the capacity fits in
// LDS; the result is identical to the multi-kernel path's.
//
// Column bitmap form (use_bm): while counting, every entry also sets the bit
// of its column in a bitmap of its row (ceil(kb/32) words per row, in the LDS
// that the staged entries use otherwise). When no bit was set twice, i.e. no
// (row, column) pair repeats, the rank of an entry within its row is the
// number of set bits below its column: an exclusive scan of the bit counts of
// all bitmap words (row-major) gives each word the block-CSR position of its
// first entry, so each entry goes straight to its position in LDS, and the
// finished arrays are copied out with coalesced stores. The scatter, the
// pairwise ranking and its scattered global stores are skipped. A repeated
// pair switches the call to the ranking path.
constexpr int kSmallThreads = 1024;
constexpr int kSmallU = 8;  // entries per thread per chunk

// Inclusive scan across the 64 lanes of a wave (shuffles, no LDS).
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T t = __shfl_up(v, off, 64);
    if (lane >= off) v += t;
  }
  return v;
}

// Exclusive scan of v[0..n) into out[0..n] (out[n] = total) by 1024 threads,
// each owning a contiguous chunk: chunk sums are scanned within each wave by
// shuffles, the 16 wave totals by one wave; wsum[] holds 16 values.
template <typename T, typename S>
__device__ void block_exscan_chunks(const S* v, int32_t n, T* out, T* wsum) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int32_t per = (n + kSmallThreads - 1) / kSmallThreads;
  const int32_t lo = min(n, tid * per), hi = min(n, lo + per);
  T sum = 0;
  for (int32_t i = lo; i < hi; ++i) sum += (T)v[i];
  const T incl = wave_incl_scan<T>(sum);
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  if (wave == 0) {
    T w = lane < kSmallThreads / 64 ? wsum[lane] : (T)0;
    w = wave_incl_scan<T>(w);
    if (lane < kSmallThreads / 64) wsum[lane] = w;
  }
  __syncthreads();
  T run = incl - sum + (wave > 0 ? wsum[wave - 1] : (T)0);
  for (int32_t i = lo; i < hi; ++i) {
    const T x = (T)v[i];
    out[i] = run;
    run += x;
  }
  if (tid == kSmallThreads - 1) out[n] = wsum[kSmallThreads / 64 - 1];
  __syncthreads();
}

__global__ __launch_bounds__(1024) void k_dyn_small(const int32_t* __restrict__ nnz_dev, int32_t max_nnz,
                                                    const int32_t* __restrict__ rows, const int32_t* __restrict__ cols,
                                                    int32_t mb, int32_t kb, int32_t GR, int32_t G, int32_t P,
                                                    int32_t* __restrict__ row_ptr, int32_t* __restrict__ col_idx,
                                                    int32_t* __restrict__ src, int32_t* __restrict__ panel_ptr,
                                                    int32_t* __restrict__ status, int32_t* __restrict__ status_out,
                                                    int32_t* __restrict__ nnz_last, int32_t use_bm) {
  extern __shared__ int64_t lds64[];
  int64_t* C = lds64;                          // [G + 1] group cost prefix
  int64_t* part64 = C + (G + 1);               // [1024]
  int32_t* cnt = (int32_t*)(part64 + kSmallThreads);  // [mb] counts, then fill positions
  int32_t* rp = cnt + mb;                      // [mb + 1]
  int32_t* part = rp + mb + 1;                 // [1024]
  int32_t* flag = part + kSmallThreads;        // [0] error, [1] nnz, [2] a (row, column) pair repeats
  uint32_t* ekey = (uint32_t*)(flag + 4);      // [max_nnz] (column << 16) | input index
  uint16_t* erow = (uint16_t*)(ekey + max_nnz); // [max_nnz] block row of each staged entry
  const int32_t wpr = (kb + 31) >> 5;
  uint32_t* bm = ekey;                         // [mb * wpr] column bitmaps (use_bm), in place of ekey/erow
  int32_t* wpos = (int32_t*)(bm + mb * wpr);   // [mb * wpr + 1] CSR position of each bitmap word's first entry (use_bm)
  uint32_t* okey = (uint32_t*)(wpos + mb * wpr + 1);  // [max_nnz] (column << 16) | input index in CSR order (use_bm)
  const int tid = threadIdx.x;
  if (tid == 0) {
    const int32_t nnz = *nnz_dev;
    flag[0] = (nnz < 0 || nnz > max_nnz) ? (int32_t)SPMM_ERR_CAPACITY : 0;
    flag[1] = nnz;
    flag[2] = 0;
  }
  for (int32_t r = tid; r < mb; r += kSmallThreads) cnt[r] = 0;
  if (use_bm)
    for (int32_t i = tid; i < mb * wpr; i += kSmallThreads) bm[i] = 0;
  __syncthreads();
  const int32_t nnz = flag[1];
  // Entries are read in chunks of kSmallU per thread, all loads of a chunk
  // issued before its LDS atomics (a load-atomic chain per entry would pay
  // the global latency once per entry). Up to kSmallThreads * kSmallU entries
  // the chunk stays in registers for the scatter pass below.
  int32_t er[kSmallU], ec[kSmallU];
  if (flag[0] == 0) {
    for (int32_t base = 0; base < nnz; base += kSmallThreads * kSmallU) {
#pragma unroll
      for (int u = 0; u < kSmallU; ++u) {
        const int32_t e = base + u * kSmallThreads + tid;
        er[u] = e < nnz ? rows[e] : 0;
        ec[u] = e < nnz ? cols[e] : 0;
      }
#pragma unroll
      for (int u = 0; u < kSmallU; ++u) {
        const int32_t e = base + u * kSmallThreads + tid;
        if (e >= nnz) continue;
        if (er[u] < 0 || er[u] >= mb || ec[u] < 0 || ec[u] >= kb) {
          atomicMax(&flag[0], (int32_t)SPMM_ERR_BAD_INDEX);
          continue;
        }
        atomicAdd(&cnt[er[u]], 1);
        if (use_bm) {
          const uint32_t bit = 1u << (ec[u] & 31);
          if (atomicOr(&bm[er[u] * wpr + (ec[u] >> 5)], bit) & bit) flag[2] = 1;
        }
      }
    }
  }
  __syncthreads();
  const int32_t err = flag[0];
  if (err) {
    if (tid == 0) {
      *status = err;
      if (status_out) *status_out = err;
    }
    return;
  }
  const bool fast = use_bm && flag[2] == 0;  // read after the barrier: the same in every thread
  const bool in_regs = nnz <= kSmallThreads * kSmallU;
  if (fast) {
    // With every (row, column) pair once, the bitmaps in row-major order list
    // block-CSR: the exclusive scan of their words' bit counts gives each word
    // the position of its first entry, and the row pointers at row starts.
    const int32_t nw = mb * wpr;
    for (int32_t i = tid; i < nw; i += kSmallThreads) wpos[i] = __popc(bm[i]);
    __syncthreads();
    block_exscan_chunks<int32_t, int32_t>(wpos, nw, wpos, part);
    for (int32_t r = tid; r <= mb; r += kSmallThreads) rp[r] = wpos[r * wpr];
    for (int32_t base = 0; base < nnz; base += kSmallThreads * kSmallU) {
      if (!in_regs) {
#pragma unroll
        for (int u = 0; u < kSmallU; ++u) {
          const int32_t e = base + u * kSmallThreads + tid;
          er[u] = e < nnz ? rows[e] : 0;
          ec[u] = e < nnz ? cols[e] : 0;
        }
      }
#pragma unroll
      for (int u = 0; u < kSmallU; ++u) {
        const int32_t e = base + u * kSmallThreads + tid;
        if (e >= nnz) continue;
        const int32_t wi = er[u] * wpr + (ec[u] >> 5);
        const int32_t pos = wpos[wi] + __popc(bm[wi] & ((1u << (ec[u] & 31)) - 1u));
        okey[pos] = ((uint32_t)ec[u] << 16) | (uint32_t)e;
      }
    }
    // block-CSR leaves LDS in order: consecutive threads write consecutive words
    __syncthreads();
    for (int32_t i = tid; i < nnz; i += kSmallThreads) {
      const uint32_t key = okey[i];
      col_idx[i] = (int32_t)(key >> 16);
      src[i] = (int32_t)(key & 0xFFFFu);
    }
  } else {
  block_exscan_chunks<int32_t, int32_t>(cnt, mb, rp, part);
  for (int32_t r = tid; r < mb; r += kSmallThreads) cnt[r] = rp[r];
  __syncthreads();
  for (int32_t base = 0; base < nnz; base += kSmallThreads * kSmallU) {
    if (!in_regs) {
#pragma unroll
      for (int u = 0; u < kSmallU; ++u) {
        const int32_t e = base + u * kSmallThreads + tid;
        er[u] = e < nnz ? rows[e] : 0;
        ec[u] = e < nnz ? cols[e] : 0;
      }
    }
#pragma unroll
    for (int u = 0; u < kSmallU; ++u) {
      const int32_t e = base + u * kSmallThreads + tid;
      if (e >= nnz) continue;
      const int32_t pos = atomicAdd(&cnt[er[u]], 1);
      ekey[pos] = ((uint32_t)ec[u] << 16) | (uint32_t)e;
      erow[pos] = (uint16_t)er[u];
    }
  }
  __syncthreads();
  // every staged entry is ranked within its row by (column, input index),
  // which is the order of the packed keys; the rank is its final position
  for (int32_t i = tid; i < nnz; i += kSmallThreads) {
    const uint32_t key = ekey[i];
    const int32_t r = erow[i];
    const int32_t lo = rp[r], hi = rp[r + 1];
    int32_t rank = 0;
    int32_t t = lo;
    for (; t + 4 <= hi; t += 4)
      rank += (ekey[t] < key) + (ekey[t + 1] < key) + (ekey[t + 2] < key) + (ekey[t + 3] < key);
    for (; t < hi; ++t) rank += ekey[t] < key;
    col_idx[lo + rank] = (int32_t)(key >> 16);
    src[lo + rank] = (int32_t)(key & 0xFFFFu);
  }
  }
  for (int32_t i = tid; i <= mb; i += kSmallThreads) row_ptr[i] = rp[i];
  // group costs (blocks + rows), their prefix, panel boundaries
  for (int32_t g = tid; g < G; g += kSmallThreads) {
    const int32_t glo = g * GR, ghi = min(mb, glo + GR);
    cnt[g] = (rp[ghi] - rp[glo]) + (ghi - glo);  // G <= mb: cnt is free again
  }
  __syncthreads();
  block_exscan_chunks<int64_t, int32_t>(cnt, G, C, part64);
  for (int32_t p = tid; p <= P; p += kSmallThreads) {
    int32_t v;
    if (p == 0) v = 0;
    else if (p == P) v = G;
    else {
      const int64_t target = ((int64_t)p * C[G]) / P;
      int32_t lo = 0, hi = G;
      while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (C[mid] >= target) hi = mid;
        else lo = mid + 1;
      }
      v = lo;
    }
    panel_ptr[p] = v;
  }
  if (tid == 0) {
    *status = 0;
    if (status_out) *status_out = 0;
    *nnz_last = nnz;
  }
}

// The end of the multi-kernel encode in one workgroup: group costs (blocks +
// rows of each group of GR block rows) from row_ptr, their exclusive scan in
// place (C[G] the total), the panel boundaries (smallest g with
// C[g] >= floor(p C[G] / P)), then the caller's status word and the entry
// count of the call. The costs and panels are skipped when the status is set.
__global__ __launch_bounds__(1024) void k_dyn_tail(const int32_t* __restrict__ row_ptr, int32_t G, int32_t GR,
                                                   int32_t mb, int32_t P, int64_t* C, int32_t* __restrict__ panel_ptr,
                                                   const int32_t* __restrict__ nnz_dev, const int32_t* status,
                                                   int32_t* __restrict__ status_out, int32_t* __restrict__ nnz_last) {
  __shared__ int64_t part64[kSmallThreads];
  const int tid = threadIdx.x;
  const int32_t st = *status;
  if (st == 0) {
    for (int32_t g = tid; g < G; g += kSmallThreads) {
      const int32_t lo = g * GR, hi = min(mb, lo + GR);
      C[g] = (int64_t)(row_ptr[hi] - row_ptr[lo]) + (hi - lo);
    }
    __syncthreads();
    block_exscan_chunks<int64_t, int64_t>(C, G, C, part64);
    for (int32_t p = tid; p <= P; p += kSmallThreads) {
      int32_t v;
      if (p == 0) v = 0;
      else if (p == P) v = G;
      else {
        const int64_t target = ((int64_t)p * C[G]) / P;
        int32_t lo = 0, hi = G;
        while (lo < hi) {
          const int32_t mid = (lo + hi) >> 1;
          if (C[mid] >= target) hi = mid;
          else lo = mid + 1;
        }
        v = lo;
      }
      panel_ptr[p] = v;
    }
  }
  if (tid == 0) {
    if (status_out) *status_out = st;
    if (nnz_last) *nnz_last = *nnz_dev;
  }
}

// LDS of the row-range encoder: kept entries' keys and rows, per-row counts.
constexpr size_t kDynRowsLdsMax = 128 * 1024;

// LDS of the one-workgroup builder; with bm_words > 0 the staged-entry region
// also holds the bitmap form's column bitmaps (bm_words words), their scanned
// bit counts (bm_words + 1) and the packed block-CSR (max_nnz words).
size_t dyn_small_lds_bytes(int32_t max_nnz, int32_t mb, int32_t G, int64_t bm_words = 0) {
  const size_t stage = sizeof(uint32_t) * (size_t)max_nnz + sizeof(uint16_t) * (size_t)max_nnz;
  const size_t region = std::max(stage, bm_words ? sizeof(uint32_t) * (2 * (size_t)bm_words + 1 + max_nnz) : 0);
  return sizeof(int64_t) * ((size_t)G + 1 + kSmallThreads) +
         sizeof(int32_t) * ((size_t)mb + mb + 1 + kSmallThreads + 4) + region;
}

// Column bitmap form: at most 32 words (1024 block columns) per row, and the
// bitmaps within the builder's LDS limit.
constexpr int32_t kBmMaxWordsPerRow = 32;

}  // namespace

constexpr size_t kDynSmallLdsMax = 64 * 1024;

// The packed keys need block columns and input indices below 2^16, the staged
// rows block rows below 2^16.
bool dynamic_small_fits(int32_t max_nnz, int32_t mb, int32_t kb, int32_t G) {
  return G <= mb && mb <= 65536 && kb <= 65536 && max_nnz <= 65536 &&
         dyn_small_lds_bytes(max_nnz, mb, G) <= kDynSmallLdsMax;
}

int32_t dyn_hist_wgs(int64_t max_nnz, int32_t mb) {
  if (mb < 1 || (int64_t)mb * (int64_t)sizeof(int32_t) > 64 * 1024) return 0;
  return (int32_t)std::min<int64_t>(256, std::max<int64_t>(1, ceil_div(max_nnz, kHistChunk)));
}

spmm_status_t build_dynamic_csr_small(const int32_t* nnz_dev, const int32_t* rows, const int32_t* cols,
                                      int32_t max_nnz, int32_t mb, int32_t kb, const Geometry& geo, PlanBuffers& pb,
                                      int32_t* status, int32_t* status_out, int32_t* nnz_last, hipStream_t s) {
  if (!dynamic_small_fits(max_nnz, mb, kb, geo.num_groups))
    return fail(SPMM_ERR_UNSUPPORTED, "dynamic capacity too large for the one-workgroup builder");
  const int64_t wpr = ((int64_t)kb + 31) / 32, bm_words = (int64_t)mb * wpr;
  const char* rank_env = getenv("SPMM_DYN_RANK");  // "pairwise": always rank by comparisons (for tests)
  const bool use_bm = !(rank_env && std::string(rank_env) == "pairwise") && wpr <= kBmMaxWordsPerRow &&
                      dyn_small_lds_bytes(max_nnz, mb, geo.num_groups, bm_words) <= kDynSmallLdsMax;
  const size_t lds = dyn_small_lds_bytes(max_nnz, mb, geo.num_groups, use_bm ? bm_words : 0);
  hipLaunchKernelGGL(k_dyn_small, dim3(1), dim3(kSmallThreads), lds, s, nnz_dev, max_nnz, rows, cols, mb, kb,
                     geo.group_rows, geo.num_groups, geo.num_panels, pb.row_ptr, pb.col_idx, pb.csr_src, pb.panel_ptr,
                     status, status_out, nnz_last, use_bm ? 1 : 0);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}



// ------------------------------------------------------------------ row-range encoder
// One launch, one workgroup per range of R block rows. Every workgroup reads
// the whole COO list (validating it, so all reach the same status), counts
// the entries above its range (its first CSR position) and keeps its own
// entries in LDS as (row in range, column, input index) keys; an entry's CSR
// place is its range's first position plus the number of kept keys below its
// own, so the rows come out in order, each in (column, input index) order, the
// canonical order of every other encoder.
// No workgroup waits for another. Panels are not built here (no product
// kernel reads them); dyn_panels derives them when a plan is exported.
constexpr int kRowsThreads = 1024;  // with kRowsU, 8192 entries in one round of loads
constexpr int kRowsU = 8;           // entries per thread loaded together

__global__ __launch_bounds__(kRowsThreads) void k_dyn_rows(const int32_t* __restrict__ nnz_dev, int32_t max_nnz,
                                                           const int32_t* __restrict__ rows,
                                                           const int32_t* __restrict__ cols, int32_t mb, int32_t kb,
                                                           int32_t R, int32_t* __restrict__ row_ptr,
                                                           int32_t* __restrict__ col_idx, int32_t* __restrict__ src,
                                                           int32_t* __restrict__ status,
                                                           int32_t* __restrict__ status_out,
                                                           int32_t* __restrict__ nnz_last) {
  extern __shared__ uint64_t rows_lds[];
  uint64_t* skey = rows_lds;                        // [max_nnz] (row in range << 53) | (column << 32) | input index
  int32_t* cnt = (int32_t*)(skey + max_nnz);        // [R + 1] entries per own row, then their offsets
  __shared__ int32_t flag[3];                       // [0] error, [1] kept entries, [2] nnz
  __shared__ int32_t wsum[kRowsThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int32_t r0 = blockIdx.x * R, nr = min(mb - r0, R);
  if (tid == 0) {
    const int32_t nnz = *nnz_dev;
    flag[0] = (nnz < 0 || nnz > max_nnz) ? (int32_t)SPMM_ERR_CAPACITY : 0;
    flag[1] = 0;
    flag[2] = nnz;
  }
  for (int32_t i = tid; i <= R; i += kRowsThreads) cnt[i] = 0;
  __syncthreads();
  const int32_t nnz = flag[2];
  int32_t above = 0;  // entries of rows before r0 seen by this thread
  if (flag[0] == 0) {
    for (int32_t base = 0; base < nnz; base += kRowsThreads * kRowsU) {
      int32_t er[kRowsU], ec[kRowsU];
#pragma unroll
      for (int u = 0; u < kRowsU; ++u) {
        const int32_t e = base + u * kRowsThreads + tid;
        er[u] = e < nnz ? rows[e] : 0;
        ec[u] = e < nnz ? cols[e] : 0;
      }
#pragma unroll
      for (int u = 0; u < kRowsU; ++u) {
        const int32_t e = base + u * kRowsThreads + tid;
        if (e >= nnz) continue;
        const int32_t r = er[u], c = ec[u];
        if (r < 0 || r >= mb || c < 0 || c >= kb) {
          atomicMax(&flag[0], (int32_t)SPMM_ERR_BAD_INDEX);
          continue;
        }
        if (r < r0) {
          ++above;
        } else if (r < r0 + nr) {
          const int32_t slot = atomicAdd(&flag[1], 1);
          skey[slot] = ((uint64_t)(uint32_t)(r - r0) << 53) | ((uint64_t)(uint32_t)c << 32) | (uint32_t)e;
          atomicAdd(&cnt[r - r0], 1);
        }
      }
    }
  }
  // the workgroup's count of entries above its rows
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) above += __shfl_xor(above, off);
  if (lane == 0) wsum[wave] = above;
  __syncthreads();
  const int32_t err = flag[0];
  if (err) {  // every workgroup read the same entries: the same status
    if (blockIdx.x == 0 && tid == 0) {
      *status = err;
      if (status_out) *status_out = err;
    }
    return;
  }
  int32_t first = 0;
#pragma unroll
  for (int w = 0; w < kRowsThreads / 64; ++w) first += wsum[w];
  // exclusive scan of the own rows' counts (R <= kRowsThreads: one per thread)
  const int32_t v = tid < nr ? cnt[tid] : 0;
  int32_t incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t t = __shfl_up(incl, off);
    if (lane >= off) incl += t;
  }
  __syncthreads();  // every thread has read cnt and the wave sums
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int32_t wpre = 0;
  for (int w = 0; w < wave; ++w) wpre += wsum[w];
  if (tid < nr) cnt[tid] = wpre + incl - v;
  if (tid == 0) cnt[nr] = flag[1];
  __syncthreads();
  for (int32_t i = tid; i < nr; i += kRowsThreads) row_ptr[r0 + i] = first + cnt[i];
  if (r0 + nr == mb && tid == 0) row_ptr[mb] = first + flag[1];
  if (blockIdx.x == 0 && tid == 0) {
    *status = 0;
    if (status_out) *status_out = 0;
    if (nnz_last) *nnz_last = nnz;
  }
  const int32_t kept = flag[1];
  if (kept <= 64) {  // one wave ranks its lanes' keys against each other, without LDS round trips
    if (tid < 64) {
      const uint64_t key = tid < kept ? skey[tid] : ~(uint64_t)0;
      const uint32_t hi = (uint32_t)(key >> 32), lo = (uint32_t)key;
      int32_t rank = 0;
      for (int32_t j = 0; j < kept; ++j) {
        const uint32_t hj = (uint32_t)__builtin_amdgcn_readlane((int)hi, j);
        const uint32_t lj = (uint32_t)__builtin_amdgcn_readlane((int)lo, j);
        rank += (hj < hi || (hj == hi && lj < lo)) ? 1 : 0;
      }
      if (tid < kept) {
        col_idx[first + rank] = (int32_t)((key >> 32) & 0x1FFFFFu);
        src[first + rank] = (int32_t)(uint32_t)key;
      }
    }
    return;
  }
  for (int32_t i = tid; i < kept; i += kRowsThreads) {
    const uint64_t key = skey[i];
    int32_t rank = 0;
#pragma unroll 8
    for (int32_t j = 0; j < kept; ++j) rank += skey[j] < key ? 1 : 0;
    col_idx[first + rank] = (int32_t)((key >> 32) & 0x1FFFFFu);
    src[first + rank] = (int32_t)(uint32_t)key;
  }
}

int32_t dyn_rows_per_wg(int32_t mb) { return std::max<int32_t>(1, std::min<int32_t>(kRowsThreads, (mb + 127) / 128)); }

size_t dyn_rows_lds_bytes(int32_t max_nnz, int32_t mb) {
  const int32_t R = dyn_rows_per_wg(mb);
  return sizeof(uint64_t) * (size_t)max_nnz + sizeof(int32_t) * (size_t)(R + 1);
}

// The key packs a row of the range in 11 bits and a block column in 21.
bool dynamic_rows_fits(int32_t max_nnz, int32_t mb, int32_t kb) {
  return max_nnz >= 1 && kb <= (1 << 21) && dyn_rows_per_wg(mb) <= 1024 &&
         dyn_rows_lds_bytes(max_nnz, mb) <= kDynRowsLdsMax;
}

spmm_status_t build_dynamic_csr_rows(const int32_t* nnz_dev, const int32_t* rows, const int32_t* cols,
                                     int32_t max_nnz, int32_t mb, int32_t kb, PlanBuffers& pb, int32_t* status,
                                     int32_t* status_out, int32_t* nnz_last, hipStream_t s) {
  if (!dynamic_rows_fits(max_nnz, mb, kb)) return fail(SPMM_ERR_UNSUPPORTED, "capacity beyond the row-range encoder");
  const int32_t R = dyn_rows_per_wg(mb);
  const size_t lds = dyn_rows_lds_bytes(max_nnz, mb);
  static bool attr_set = false;
  if (!attr_set) {
    SPMM_HIP(hipFuncSetAttribute((const void*)k_dyn_rows, hipFuncAttributeMaxDynamicSharedMemorySize, kDynRowsLdsMax));
    attr_set = true;
  }
  hipLaunchKernelGGL(k_dyn_rows, dim3((unsigned)ceil_div(mb, R)), dim3(kRowsThreads), lds, s, nnz_dev, max_nnz, rows,
                     cols, mb, kb, R, pb.row_ptr, pb.col_idx, pb.csr_src, status, status_out, nnz_last);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

spmm_status_t dyn_panels(const Geometry& geo, int32_t mb, PlanBuffers& pb, const int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(k_dyn_tail, dim3(1), dim3(kSmallThreads), 0, s, pb.row_ptr, geo.num_groups, geo.group_rows, mb,
                     geo.num_panels, pb.cost_prefix, pb.panel_ptr, (const int32_t*)nullptr, status, (int32_t*)nullptr,
                     (int32_t*)nullptr);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

spmm_status_t build_dynamic_csr(const int32_t* nnz_dev, const int32_t* rows, const int32_t* cols, int32_t max_nnz,
                                int32_t mb, int32_t kb, int32_t b, int32_t k, const Geometry& geo, PlanBuffers& pb,
                                const void* vals, void* vals_out, int elem_bytes, const float* scales,
                                float* scales_out, int32_t* status, int32_t* status_out, int32_t* nnz_last,
                                hipStream_t s) {
  if (mb > 1024 * 64) return fail(SPMM_ERR_UNSUPPORTED, "dynamic CSR builder supports at most 65536 block rows");
  int32_t* row_cnt = pb.scratch;            // [mb]
  int32_t* fill = pb.scratch + mb;          // [mb]
  int32_t* tmp_col = pb.tmp_col;            // [max_nnz] scratch for the row sort
  int32_t* tmp_src = pb.tmp_src;
  hipLaunchKernelGGL(k_dyn_zero, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(256, ceil_div(2 * mb, 256)))),
                     dim3(256), 0, s, row_cnt, (int64_t)2 * mb, status);
  const int32_t wgs = dyn_hist_wgs(max_nnz, mb);
  if (pb.hist && wgs > 0 && wgs <= pb.hist_wgs && !(getenv("SPMM_DYN_HIST") && getenv("SPMM_DYN_HIST")[0] == '0')) {
    // counting sort by block row, no global atomics
    const int32_t chunk = (int32_t)ceil_div(std::max(max_nnz, 1), wgs);
    const size_t lds = sizeof(int32_t) * (size_t)mb;
    hipLaunchKernelGGL(k_dyn_hist, dim3((unsigned)wgs), dim3(256), lds, s, nnz_dev, max_nnz, rows, cols, mb, kb, chunk,
                       pb.hist, status);
    hipLaunchKernelGGL(k_dyn_hist_scan, dim3((unsigned)ceil_div(mb, 256)), dim3(256), 0, s, pb.hist, wgs, mb, row_cnt,
                       status);
    hipLaunchKernelGGL(k_dyn_scan_rows, dim3(1), dim3(1024), 0, s, row_cnt, mb, pb.row_ptr, status);
    hipLaunchKernelGGL(k_dyn_hist_scatter, dim3((unsigned)wgs), dim3(256), lds, s, nnz_dev, rows, cols, mb, chunk,
                       pb.hist, pb.row_ptr, pb.col_idx, pb.csr_src, status);
  } else {
    const unsigned egrid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(2048, ceil_div(max_nnz, 256)));
    hipLaunchKernelGGL(k_dyn_row_count, dim3(egrid), dim3(256), 0, s, nnz_dev, max_nnz, rows, cols, mb, kb, row_cnt,
                       status);
    hipLaunchKernelGGL(k_dyn_scan_rows, dim3(1), dim3(1024), 0, s, row_cnt, mb, pb.row_ptr, status);
    hipLaunchKernelGGL(k_dyn_row_scatter, dim3(egrid), dim3(256), 0, s, nnz_dev, rows, cols, pb.row_ptr, fill,
                       pb.col_idx, pb.csr_src, status);
  }
  hipLaunchKernelGGL(k_dyn_row_sort, dim3((unsigned)mb), dim3(256), 0, s, pb.row_ptr, pb.col_idx, pb.csr_src, tmp_col,
                     tmp_src, kb, status);
  if (vals_out && max_nnz > 0) {
    const unsigned vgrid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, ceil_div((int64_t)max_nnz * b * b, 1024)));
    if (elem_bytes == 1)
      hipLaunchKernelGGL(k_dyn_gather<uint8_t>, dim3(vgrid), dim3(256), 0, s, nnz_dev, pb.csr_src, pb.col_idx, b, k,
                         (const uint8_t*)vals, (uint8_t*)vals_out, scales, scales_out, status);
    else if (elem_bytes == 2)
      hipLaunchKernelGGL(k_dyn_gather<uint16_t>, dim3(vgrid), dim3(256), 0, s, nnz_dev, pb.csr_src, pb.col_idx, b, k,
                         (const uint16_t*)vals, (uint16_t*)vals_out, scales, scales_out, status);
    else
      hipLaunchKernelGGL(k_dyn_gather<uint32_t>, dim3(vgrid), dim3(256), 0, s, nnz_dev, pb.csr_src, pb.col_idx, b, k,
                         (const uint32_t*)vals, (uint32_t*)vals_out, scales, scales_out, status);
  }
  hipLaunchKernelGGL(k_dyn_tail, dim3(1), dim3(kSmallThreads), 0, s, pb.row_ptr, geo.num_groups, geo.group_rows, mb,
                     geo.num_panels, pb.cost_prefix, pb.panel_ptr, nnz_dev, status, status_out, nnz_last);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

}  // namespace spmm
