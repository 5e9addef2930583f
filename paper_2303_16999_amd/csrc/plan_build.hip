// GPU plan builder: block mask (static) or COO list (dynamic) -> the bucketed
// layout the compute kernels walk, plus the canonical block-CSR and the
// cost-balanced panels.
//
// The paper's static partitioner balances the known nonzeros over the parts
// it creates (Section 3.2); the dynamic mode re-buckets indices and values on
// every run into buckets sized from the maximum density (Section 3.3,
// Appendix A.2). Both are done here with integer-only, deterministic kernels:
// counts, exclusive scans, ballot compaction and per-cell sorts, so the result
// does not depend on thread timing.
#include "common.h"

namespace spmm {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Block-wide exclusive scan of one int per thread; returns the block total.
template <typename T>
__device__ T block_exscan(T v, T* sh, T& total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    T add = tid >= off ? sh[tid - off] : T(0);
    __syncthreads();
    sh[tid] += add;
    __syncthreads();
  }
  T incl = sh[tid];
  total = sh[blockDim.x - 1];
  __syncthreads();
  return incl - v;
}

__global__ void k_scan_reduce(const int32_t* __restrict__ in, int64_t n, int32_t* __restrict__ partials,
                              const int32_t* status) {
  if (status && *status) return;
  __shared__ int32_t sh[kScanThreads];
  int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int32_t s = 0;
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += in[base + i];
  int32_t tot;
  block_exscan<int32_t>(s, sh, tot);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// One block scans the per-tile partials in place (exclusive), carrying across
// passes of kScanThreads entries, and writes the grand total to out[n].
__global__ void k_scan_partials(int32_t* __restrict__ partials, int64_t nparts, int32_t* __restrict__ out,
                                int64_t n, const int32_t* status) {
  if (status && *status) return;
  __shared__ int32_t sh[kScanThreads];
  int32_t carry = 0;
  for (int64_t b = 0; b < nparts; b += kScanThreads) {
    int64_t i = b + threadIdx.x;
    int32_t v = i < nparts ? partials[i] : 0;
    int32_t tot;
    int32_t ex = block_exscan<int32_t>(v, sh, tot);
    if (i < nparts) partials[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) out[n] = carry;
}

__global__ void k_scan_apply(const int32_t* __restrict__ in, int64_t n, const int32_t* __restrict__ partials,
                             int32_t* __restrict__ out, const int32_t* status) {
  if (status && *status) return;
  __shared__ int32_t sh[kScanThreads];
  int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int32_t v[kScanItems];
  int32_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? in[base + i] : 0;
    s += v[i];
  }
  int32_t tot;
  int32_t run = block_exscan<int32_t>(s, sh, tot) + partials[blockIdx.x];
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
}

// out[0..n] = exclusive prefix sums of in[0..n); out[n] = total. `partials`
// needs ceil(n / kScanTile) ints. in and out may alias.
spmm_status_t exscan_i32(const int32_t* in, int32_t* out, int64_t n, int32_t* partials, const int32_t* status,
                         hipStream_t s) {
  int64_t nparts = ceil_div(n, kScanTile);
  if (nparts == 0) {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, out, (int64_t)1, 0);
    return hipGetLastError() == hipSuccess ? SPMM_OK : fail(SPMM_ERR_HIP, "scan launch failed");
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nparts), dim3(kScanThreads), 0, s, in, n, partials, status);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, s, partials, nparts, out, n, status);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nparts), dim3(kScanThreads), 0, s, in, n, partials, out, status);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPMM_OK : fail_hip(e, "scan launch");
}

__device__ __forceinline__ int64_t cell_of(int32_t r, int32_t c, int32_t GR, int32_t CW, int32_t NCH) {
  int32_t g = r / GR, lr = r - g * GR, ch = c / CW;
  return ((int64_t)g * NCH + ch) * GR + lr;
}

// ------------------------------------------------------------------ static: mask -> counts
// One wave per block row; columns are visited in strips of 64, and a chunk of
// CW columns (a power of two <= 64) never straddles a strip.
__global__ void k_static_count(const uint8_t* __restrict__ mask, int32_t mb, int32_t kb, int32_t GR, int32_t CW,
                               int32_t NCH, int32_t* __restrict__ row_cnt, int32_t* __restrict__ cell_cnt) {
  const int lane = threadIdx.x & 63;
  const int32_t r = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (r >= mb) return;
  const uint8_t* row = mask + (int64_t)r * kb;
  int32_t total = 0;
  for (int32_t c0 = 0; c0 < kb; c0 += 64) {
    int32_t c = c0 + lane;
    bool nz = c < kb && row[c] != 0;
    uint64_t bal = __ballot(nz);
    total += __popcll(bal);
    // lane q < 64/CW reports chunk q of this strip
    int32_t ch_local = lane;
    int32_t ch = c0 / CW + ch_local;
    if (ch_local < 64 / CW && ch * CW < kb) {
      uint64_t cm = (CW == 64) ? ~0ull : (((1ull << CW) - 1) << (ch_local * CW));
      cell_cnt[cell_of(r, ch * CW, GR, CW, NCH)] = __popcll(bal & cm);
    }
  }
  if (lane == 0) row_cnt[r] = total;
}

__global__ void k_static_fill(const uint8_t* __restrict__ mask, int32_t mb, int32_t kb, int32_t GR, int32_t CW,
                              int32_t NCH, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ cell_ptr,
                              int32_t* __restrict__ col_idx, int32_t* __restrict__ ent_col,
                              int32_t* __restrict__ ent_src) {
  const int lane = threadIdx.x & 63;
  const int32_t r = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (r >= mb) return;
  const uint8_t* row = mask + (int64_t)r * kb;
  const uint64_t lt = (1ull << lane) - 1;
  int32_t run = row_ptr[r];
  for (int32_t c0 = 0; c0 < kb; c0 += 64) {
    int32_t c = c0 + lane;
    bool nz = c < kb && row[c] != 0;
    uint64_t bal = __ballot(nz);
    if (nz) {
      int32_t csr = run + __popcll(bal & lt);
      col_idx[csr] = c;
      int32_t first = (c / CW) * CW - c0;  // first lane of this chunk in the strip
      uint64_t from = first > 0 ? ~((1ull << first) - 1) : ~0ull;
      int32_t e = cell_ptr[cell_of(r, c, GR, CW, NCH)] + __popcll(bal & lt & from);
      ent_col[e] = c;
      ent_src[e] = csr;
    }
    run += __popcll(bal);
  }
}

// ------------------------------------------------------------------ groups and panels
__global__ void k_group_cost(const int32_t* __restrict__ cell_ptr, int32_t G, int32_t NCH, int32_t GR, int32_t mb,
                             int64_t* __restrict__ cost, const int32_t* status) {
  if (status && *status) return;
  int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  int64_t lo = (int64_t)g * NCH * GR, hi = (int64_t)(g + 1) * NCH * GR;
  int32_t rows = min(GR, mb - g * GR);
  cost[g] = (int64_t)(cell_ptr[hi] - cell_ptr[lo]) + rows;
}

// In-place exclusive scan of G int64 costs into C[0..G] (C[G] = total); one block.
__global__ void k_cost_scan(int64_t* __restrict__ C, int32_t G, const int32_t* status) {
  if (status && *status) return;
  __shared__ int64_t sh[kScanThreads];
  int64_t carry = 0;
  for (int32_t b = 0; b < G; b += kScanThreads) {
    int32_t i = b + threadIdx.x;
    int64_t v = i < G ? C[i] : 0;
    int64_t tot;
    int64_t ex = block_exscan<int64_t>(v, sh, tot);
    if (i < G) C[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) C[G] = carry;
}

// panel_ptr[p] = smallest g in [0, G] with C[g] >= floor(p * C[G] / P).
__global__ void k_panels(const int64_t* __restrict__ C, int32_t G, int32_t P, int32_t* __restrict__ panel_ptr,
                         const int32_t* status) {
  if (status && *status) return;
  int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > P) return;
  if (p == 0) { panel_ptr[0] = 0; return; }
  if (p == P) { panel_ptr[P] = G; return; }
  int64_t target = ((int64_t)p * C[G]) / P;
  int32_t lo = 0, hi = G;  // answer in [lo, hi]
  while (lo < hi) {
    int32_t mid = (lo + hi) >> 1;
    if (C[mid] >= target) hi = mid; else lo = mid + 1;
  }
  panel_ptr[p] = lo;
}

}  // namespace


namespace {

spmm_status_t build_panels(const Geometry& geo, int32_t mb, PlanBuffers& pb, const int32_t* status, hipStream_t s) {
  const int32_t G = geo.num_groups;
  hipLaunchKernelGGL(k_group_cost, dim3((unsigned)ceil_div(G, 256)), dim3(256), 0, s, pb.cell_ptr, G,
                     geo.num_chunks, geo.group_rows, mb, pb.cost_prefix, status);
  hipLaunchKernelGGL(k_cost_scan, dim3(1), dim3(kScanThreads), 0, s, pb.cost_prefix, G, status);
  hipLaunchKernelGGL(k_panels, dim3((unsigned)ceil_div(geo.num_panels + 1, 256)), dim3(256), 0, s, pb.cost_prefix,
                     G, geo.num_panels, pb.panel_ptr, status);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPMM_OK : fail_hip(e, "panel launch");
}

// ------------------------------------------------------------------ dynamic
__global__ void k_dyn_count(const int32_t* __restrict__ nnz_dev, int32_t max_nnz, const int32_t* __restrict__ rows,
                            const int32_t* __restrict__ cols, int32_t mb, int32_t kb, int32_t GR, int32_t CW,
                            int32_t NCH, int32_t* __restrict__ cell_cnt, int32_t* __restrict__ status) {
  const int32_t nnz = *nnz_dev;
  if (nnz < 0 || nnz > max_nnz) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicMax(status, (int32_t)SPMM_ERR_CAPACITY);
    return;
  }
  for (int32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += gridDim.x * blockDim.x) {
    int32_t r = rows[e], c = cols[e];
    if (r < 0 || r >= mb || c < 0 || c >= kb) {
      atomicMax(status, (int32_t)SPMM_ERR_BAD_INDEX);
      continue;
    }
    atomicAdd(&cell_cnt[cell_of(r, c, GR, CW, NCH)], 1);
  }
}

__global__ void k_dyn_scatter(const int32_t* __restrict__ nnz_dev, const int32_t* __restrict__ rows,
                              const int32_t* __restrict__ cols, int32_t GR, int32_t CW, int32_t NCH,
                              const int32_t* __restrict__ cell_ptr, int32_t* __restrict__ fill,
                              int32_t* __restrict__ ent_col, int32_t* __restrict__ ent_src,
                              const int32_t* __restrict__ status) {
  if (*status) return;
  const int32_t nnz = *nnz_dev;
  for (int32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += gridDim.x * blockDim.x) {
    int32_t r = rows[e], c = cols[e];
    int64_t cell = cell_of(r, c, GR, CW, NCH);
    int32_t pos = cell_ptr[cell] + atomicAdd(&fill[cell], 1);
    ent_col[pos] = c;
    ent_src[pos] = e;
  }
}

// Each cell's entries are few (at most CW distinct columns plus duplicates):
// one thread sorts its cell by (column, source index), which makes the result
// independent of the order the scatter's atomics handed out slots.
__global__ void k_dyn_sort_cells(const int32_t* __restrict__ cell_ptr, int64_t ncell, int32_t* __restrict__ ent_col,
                                 int32_t* __restrict__ ent_src, const int32_t* __restrict__ status) {
  if (*status) return;
  for (int64_t cidx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; cidx < ncell;
       cidx += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = cell_ptr[cidx], hi = cell_ptr[cidx + 1];
    for (int32_t i = lo + 1; i < hi; ++i) {
      int32_t kc = ent_col[i], ks = ent_src[i];
      int32_t j = i - 1;
      while (j >= lo && (ent_col[j] > kc || (ent_col[j] == kc && ent_src[j] > ks))) {
        ent_col[j + 1] = ent_col[j];
        ent_src[j + 1] = ent_src[j];
        --j;
      }
      ent_col[j + 1] = kc;
      ent_src[j + 1] = ks;
    }
  }
}

__global__ void k_status_out(const int32_t* __restrict__ internal, int32_t* __restrict__ out) {
  if (threadIdx.x == 0) *out = *internal;
}

// CSR of a bucketed plan: one wave per block row walks the row's cells in
// chunk order (columns ascend across chunks and inside each cell).
__global__ void k_row_counts_from_cells(const int32_t* __restrict__ cell_ptr, int32_t mb, int32_t GR, int32_t NCH,
                                        int32_t* __restrict__ row_cnt, const int32_t* status) {
  if (status && *status) return;
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= mb) return;
  int32_t g = r / GR, lr = r - g * GR, s = 0;
  for (int32_t ch = 0; ch < NCH; ++ch) {
    int64_t cidx = ((int64_t)g * NCH + ch) * GR + lr;
    s += cell_ptr[cidx + 1] - cell_ptr[cidx];
  }
  row_cnt[r] = s;
}

__global__ void k_csr_from_cells(const int32_t* __restrict__ cell_ptr, const int32_t* __restrict__ ent_col,
                                 const int32_t* __restrict__ ent_src, int32_t mb, int32_t GR, int32_t NCH,
                                 const int32_t* __restrict__ row_ptr, int32_t* __restrict__ col_idx,
                                 int32_t* __restrict__ csr_src, const int32_t* status) {
  if (status && *status) return;
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= mb) return;
  int32_t g = r / GR, lr = r - g * GR, out = row_ptr[r];
  for (int32_t ch = 0; ch < NCH; ++ch) {
    int64_t cidx = ((int64_t)g * NCH + ch) * GR + lr;
    for (int32_t e = cell_ptr[cidx]; e < cell_ptr[cidx + 1]; ++e, ++out) {
      col_idx[out] = ent_col[e];
      csr_src[out] = ent_src[e];
    }
  }
}

template <typename T>
__global__ void k_pack(const int32_t* __restrict__ ent_src, const int32_t* __restrict__ ent_col, int64_t nnz,
                       int32_t b, int32_t k, const T* __restrict__ src, T* __restrict__ dst,
                       const float* __restrict__ ssrc, float* __restrict__ sdst) {
  const int64_t bb = (int64_t)b * b;
  const int32_t krem = k - (k / b) * b;  // columns of the last block column inside the matrix (0 = full)
  const int32_t kb_last = (k + b - 1) / b - 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nnz * bb; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t e = i / bb, w = i - e * bb;
    int32_t col = (int32_t)(w % b);
    T v = src[(int64_t)ent_src[e] * bb + w];
    if (krem && ent_col[e] == kb_last && col >= krem) v = T(0);
    dst[i] = v;
    if (w == 0 && ssrc) sdst[e] = ssrc[ent_src[e]];
  }
}

template <typename T>
__global__ void k_pack_dyn(const int32_t* __restrict__ ent_src, const int32_t* __restrict__ ent_col,
                           const int32_t* __restrict__ nnz_dev, int32_t b, int32_t k, const T* __restrict__ src,
                           T* __restrict__ dst, const float* __restrict__ ssrc, float* __restrict__ sdst,
                           const int32_t* __restrict__ status) {
  if (*status) return;
  const int64_t nnz = *nnz_dev;
  const int64_t bb = (int64_t)b * b;
  const int32_t krem = k - (k / b) * b;
  const int32_t kb_last = (k + b - 1) / b - 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nnz * bb; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t e = i / bb, w = i - e * bb;
    int32_t col = (int32_t)(w % b);
    T v = src[(int64_t)ent_src[e] * bb + w];
    if (krem && ent_col[e] == kb_last && col >= krem) v = T(0);
    dst[i] = v;
    if (w == 0 && ssrc) sdst[e] = ssrc[ent_src[e]];
  }
}

// Largest block count of one (group, chunk): cells of a chunk are contiguous.
__global__ void k_max_chunk(const int32_t* __restrict__ cell_ptr, int64_t nchunks_total, int32_t GR,
                            int32_t* __restrict__ out) {
  int32_t best = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nchunks_total; i += (int64_t)gridDim.x * blockDim.x)
    best = max(best, cell_ptr[(i + 1) * GR] - cell_ptr[i * GR]);
  atomicMax(out, best);
}

__global__ void k_chunk_overflow(const int32_t* __restrict__ cell_ptr, int64_t nchunks_total, int32_t GR,
                                 int32_t wcap, const int32_t* __restrict__ status, int32_t* __restrict__ ovf) {
  if (*status) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nchunks_total; i += (int64_t)gridDim.x * blockDim.x)
    if (cell_ptr[(i + 1) * GR] - cell_ptr[i * GR] > wcap) atomicOr(ovf, 1);
}

// Values in block-CSR order, zeroing the part of edge blocks beyond column k.
template <typename T>
__global__ void k_copy_csr(const int32_t* __restrict__ col_idx, int64_t nnz, int32_t b, int32_t k,
                           const T* __restrict__ src, T* __restrict__ dst, const float* __restrict__ ssrc,
                           float* __restrict__ sdst) {
  const int64_t bb = (int64_t)b * b;
  const int32_t krem = k - (k / b) * b;
  const int32_t kb_last = (k + b - 1) / b - 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nnz * bb; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t e = i / bb, w = i - e * bb;
    T v = src[i];
    if (krem && col_idx[e] == kb_last && (int32_t)(w % b) >= krem) v = T(0);
    dst[i] = v;
    if (w == 0 && ssrc) sdst[e] = ssrc[e];
  }
}

}  // namespace

spmm_status_t copy_values_csr(const int32_t* col_idx, int64_t nnz, int32_t b, int32_t k, const void* src, void* dst,
                              int elem_bytes, const float* ssrc, float* sdst, hipStream_t s) {
  if (nnz == 0) return SPMM_OK;
  const int64_t total = nnz * (int64_t)b * b;
  unsigned grid = (unsigned)std::min<int64_t>(8192, ceil_div(total, 256));
  if (elem_bytes == 1)
    hipLaunchKernelGGL(k_copy_csr<uint8_t>, dim3(grid), dim3(256), 0, s, col_idx, nnz, b, k, (const uint8_t*)src,
                       (uint8_t*)dst, ssrc, sdst);
  else if (elem_bytes == 2)
    hipLaunchKernelGGL(k_copy_csr<uint16_t>, dim3(grid), dim3(256), 0, s, col_idx, nnz, b, k, (const uint16_t*)src,
                       (uint16_t*)dst, ssrc, sdst);
  else
    hipLaunchKernelGGL(k_copy_csr<uint32_t>, dim3(grid), dim3(256), 0, s, col_idx, nnz, b, k, (const uint32_t*)src,
                       (uint32_t*)dst, ssrc, sdst);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

spmm_status_t chunk_overflow_flag(const KernelPlan& kp, int32_t wcap, const int32_t* status, int32_t* ovf,
                                  hipStream_t s) {
  const int64_t total = (int64_t)kp.num_groups * kp.num_chunks;
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, ovf, (int64_t)1, 0);
  unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, ceil_div(total, 256)));
  hipLaunchKernelGGL(k_chunk_overflow, dim3(grid), dim3(256), 0, s, kp.cell_ptr, total, kp.group_rows, wcap, status, ovf);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

spmm_status_t pack_values_dyn(const KernelPlan& kp, int64_t max_nnz, const int32_t* nnz_dev, const void* src,
                              void* dst, int elem_bytes, const float* ssrc, float* sdst, const int32_t* status,
                              hipStream_t s) {
  if (max_nnz == 0) return SPMM_OK;
  const int64_t total = max_nnz * (int64_t)kp.b * kp.b;
  unsigned grid = (unsigned)std::min<int64_t>(4096, ceil_div(total, 256 * 4));
  if (elem_bytes == 1)
    hipLaunchKernelGGL(k_pack_dyn<uint8_t>, dim3(grid), dim3(256), 0, s, kp.ent_src, kp.ent_col, nnz_dev, kp.b, kp.k,
                       (const uint8_t*)src, (uint8_t*)dst, ssrc, sdst, status);
  else if (elem_bytes == 2)
    hipLaunchKernelGGL(k_pack_dyn<uint16_t>, dim3(grid), dim3(256), 0, s, kp.ent_src, kp.ent_col, nnz_dev, kp.b, kp.k,
                       (const uint16_t*)src, (uint16_t*)dst, ssrc, sdst, status);
  else
    hipLaunchKernelGGL(k_pack_dyn<uint32_t>, dim3(grid), dim3(256), 0, s, kp.ent_src, kp.ent_col, nnz_dev, kp.b, kp.k,
                       (const uint32_t*)src, (uint32_t*)dst, ssrc, sdst, status);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

spmm_status_t max_chunk_blocks(const KernelPlan& kp, int32_t* scratch_dev, int32_t* out_host, hipStream_t s) {
  const int64_t total = (int64_t)kp.num_groups * kp.num_chunks;
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, scratch_dev, (int64_t)1, 0);
  unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, ceil_div(total, 256)));
  hipLaunchKernelGGL(k_max_chunk, dim3(grid), dim3(256), 0, s, kp.cell_ptr, total, kp.group_rows, scratch_dev);
  SPMM_HIP(hipGetLastError());
  SPMM_HIP(hipMemcpyAsync(out_host, scratch_dev, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  SPMM_HIP(hipStreamSynchronize(s));
  return SPMM_OK;
}

spmm_status_t build_static_plan(const uint8_t* mask_dev, int32_t mb, int32_t kb, const Geometry& geo,
                                PlanBuffers& pb, hipStream_t s) {
  const int32_t GR = geo.group_rows, CW = geo.chunk_cols, NCH = geo.num_chunks;
  const int64_t ncell = geo.num_cells;
  int32_t* row_cnt = pb.scratch;                 // [mb]
  int32_t* partials = pb.scratch + mb;           // scan partials
  hipLaunchKernelGGL(k_fill_i32, dim3(256), dim3(256), 0, s, pb.cell_ptr, ncell + 1, 0);
  const int rows_per_block = 4;
  dim3 grid((unsigned)ceil_div(mb, rows_per_block)), block(64 * rows_per_block);
  hipLaunchKernelGGL(k_static_count, grid, block, 0, s, mask_dev, mb, kb, GR, CW, NCH, row_cnt, pb.cell_ptr);
  spmm_status_t st = exscan_i32(row_cnt, pb.row_ptr, mb, partials, nullptr, s);
  if (st != SPMM_OK) return st;
  st = exscan_i32(pb.cell_ptr, pb.cell_ptr, ncell, partials, nullptr, s);
  if (st != SPMM_OK) return st;
  hipLaunchKernelGGL(k_static_fill, grid, block, 0, s, mask_dev, mb, kb, GR, CW, NCH, pb.row_ptr, pb.cell_ptr,
                     pb.col_idx, pb.ent_col, pb.ent_src);
  SPMM_HIP(hipGetLastError());
  return build_panels(geo, mb, pb, nullptr, s);
}

spmm_status_t build_dynamic_plan(const int32_t* nnz_dev, const int32_t* rows, const int32_t* cols, int32_t max_nnz,
                                 int32_t mb, int32_t kb, const Geometry& geo, PlanBuffers& pb,
                                 int32_t* status_internal, int32_t* status_out, hipStream_t s) {
  const int32_t GR = geo.group_rows, CW = geo.chunk_cols, NCH = geo.num_chunks;
  const int64_t ncell = geo.num_cells;
  int32_t* fill = pb.scratch;                    // [ncell]
  int32_t* partials = pb.scratch + ncell;        // scan partials
  unsigned zgrid = (unsigned)std::min<int64_t>(1024, ceil_div(ncell + 1, 256));
  hipLaunchKernelGGL(k_fill_i32, dim3(zgrid), dim3(256), 0, s, pb.cell_ptr, ncell + 1, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(zgrid), dim3(256), 0, s, fill, ncell, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, status_internal, (int64_t)1, 0);
  unsigned egrid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(2048, ceil_div(max_nnz, 256)));
  hipLaunchKernelGGL(k_dyn_count, dim3(egrid), dim3(256), 0, s, nnz_dev, max_nnz, rows, cols, mb, kb, GR, CW, NCH,
                     pb.cell_ptr, status_internal);
  spmm_status_t st = exscan_i32(pb.cell_ptr, pb.cell_ptr, ncell, partials, status_internal, s);
  if (st != SPMM_OK) return st;
  hipLaunchKernelGGL(k_dyn_scatter, dim3(egrid), dim3(256), 0, s, nnz_dev, rows, cols, GR, CW, NCH, pb.cell_ptr, fill,
                     pb.ent_col, pb.ent_src, status_internal);
  unsigned cgrid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, ceil_div(ncell, 256)));
  hipLaunchKernelGGL(k_dyn_sort_cells, dim3(cgrid), dim3(256), 0, s, pb.cell_ptr, ncell, pb.ent_col, pb.ent_src,
                     status_internal);
  st = build_panels(geo, mb, pb, status_internal, s);
  if (st != SPMM_OK) return st;
  if (status_out) hipLaunchKernelGGL(k_status_out, dim3(1), dim3(64), 0, s, status_internal, status_out);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

spmm_status_t dynamic_csr_from_cells(int32_t mb, const Geometry& geo, PlanBuffers& pb, const int32_t* status,
                                     hipStream_t s) {
  int32_t* row_cnt = pb.scratch;
  int32_t* partials = pb.scratch + mb;
  dim3 grid((unsigned)ceil_div(mb, 256)), block(256);
  hipLaunchKernelGGL(k_row_counts_from_cells, grid, block, 0, s, pb.cell_ptr, mb, geo.group_rows, geo.num_chunks,
                     row_cnt, status);
  spmm_status_t st = exscan_i32(row_cnt, pb.row_ptr, mb, partials, status, s);
  if (st != SPMM_OK) return st;
  hipLaunchKernelGGL(k_csr_from_cells, grid, block, 0, s, pb.cell_ptr, pb.ent_col, pb.ent_src, mb, geo.group_rows,
                     geo.num_chunks, pb.row_ptr, pb.col_idx, pb.csr_src, status);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

spmm_status_t pack_values(const KernelPlan& kp, int64_t nnz, const void* src, void* dst, int elem_bytes,
                          const float* ssrc, float* sdst, hipStream_t s) {
  if (nnz == 0) return SPMM_OK;
  const int64_t total = nnz * (int64_t)kp.b * kp.b;
  unsigned grid = (unsigned)std::min<int64_t>(8192, ceil_div(total, 256));
  if (elem_bytes == 1)
    hipLaunchKernelGGL(k_pack<uint8_t>, dim3(grid), dim3(256), 0, s, kp.ent_src, kp.ent_col, nnz, kp.b, kp.k,
                       (const uint8_t*)src, (uint8_t*)dst, ssrc, sdst);
  else if (elem_bytes == 2)
    hipLaunchKernelGGL(k_pack<uint16_t>, dim3(grid), dim3(256), 0, s, kp.ent_src, kp.ent_col, nnz, kp.b, kp.k,
                       (const uint16_t*)src, (uint16_t*)dst, ssrc, sdst);
  else
    hipLaunchKernelGGL(k_pack<uint32_t>, dim3(grid), dim3(256), 0, s, kp.ent_src, kp.ent_col, nnz, kp.b, kp.k,
                       (const uint32_t*)src, (uint32_t*)dst, ssrc, sdst);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

}  // namespace spmm
