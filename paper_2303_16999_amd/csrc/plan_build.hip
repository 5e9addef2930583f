// GPU static plan builder: block mask -> block-CSR, the cost-balanced panels
// of the row groups and the in-group column-major order, plus the value copy
// into the plan.
//
// The paper's static partitioner balances the known nonzeros over the parts
// it creates (Section 3.2). Here that is done with integer-only,
// deterministic kernels (counts, exclusive scans, ballot compaction, LDS
// histograms), so the result does not depend on thread timing and equals the
// CPU derivation bit for bit. The dynamic mode's encoder is in dyn_csr.hip.
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

// ------------------------------------------------------------------ static: mask -> block-CSR
// One wave per block row; columns are visited in strips of 64.
__global__ void k_static_count(const uint8_t* __restrict__ mask, int32_t mb, int32_t kb,
                               int32_t* __restrict__ row_cnt) {
  const int lane = threadIdx.x & 63;
  const int32_t r = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (r >= mb) return;
  const uint8_t* row = mask + (int64_t)r * kb;
  int32_t total = 0;
  for (int32_t c0 = 0; c0 < kb; c0 += 64) {
    const int32_t c = c0 + lane;
    total += __popcll(__ballot(c < kb && row[c] != 0));
  }
  if (lane == 0) row_cnt[r] = total;
}

__global__ void k_static_fill(const uint8_t* __restrict__ mask, int32_t mb, int32_t kb,
                              const int32_t* __restrict__ row_ptr, int32_t* __restrict__ col_idx) {
  const int lane = threadIdx.x & 63;
  const int32_t r = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (r >= mb) return;
  const uint8_t* row = mask + (int64_t)r * kb;
  const uint64_t lt = (1ull << lane) - 1;
  int32_t run = row_ptr[r];
  for (int32_t c0 = 0; c0 < kb; c0 += 64) {
    const int32_t c = c0 + lane;
    const bool nz = c < kb && row[c] != 0;
    const uint64_t bal = __ballot(nz);
    if (nz) col_idx[run + __popcll(bal & lt)] = c;
    run += __popcll(bal);
  }
}

// ------------------------------------------------------------------ in-group column-major order
// One workgroup per row group lists the group's blocks by (block column, block
// row). Block columns are taken in windows of kOrderWin: per window the
// workgroup counts the group's blocks of each column in LDS, scans the counts
// into first slots, then places the group's rows one after another, so that
// blocks of one column keep ascending rows. A mask holds a column at most once
// per row, so the threads placing one row never share a counter.
constexpr int kOrderThreads = 256;
constexpr int kOrderWin = 4096;
constexpr int kOrderPer = kOrderWin / kOrderThreads;

__global__ __launch_bounds__(kOrderThreads) void k_group_order(const int32_t* __restrict__ row_ptr,
                                                               const int32_t* __restrict__ col_idx, int32_t mb,
                                                               int32_t kb, int32_t GR, int32_t* __restrict__ order) {
  __shared__ int32_t cnt[kOrderWin];
  __shared__ int32_t sh[kOrderThreads];
  const int tid = threadIdx.x;
  const int32_t r_lo = blockIdx.x * GR, r_hi = min(mb, r_lo + GR);
  const int32_t q_lo = row_ptr[r_lo], q_hi = row_ptr[r_hi];
  int32_t base = q_lo;
  for (int32_t w0 = 0; w0 < kb; w0 += kOrderWin) {
    for (int i = tid; i < kOrderWin; i += kOrderThreads) cnt[i] = 0;
    __syncthreads();
    for (int32_t q = q_lo + tid; q < q_hi; q += kOrderThreads) {
      const int32_t c = col_idx[q] - w0;
      if (c >= 0 && c < kOrderWin) atomicAdd(&cnt[c], 1);
    }
    __syncthreads();
    int32_t v[kOrderPer], s = 0;
#pragma unroll
    for (int i = 0; i < kOrderPer; ++i) {
      v[i] = cnt[tid * kOrderPer + i];
      s += v[i];
    }
    int32_t tot;
    int32_t run = block_exscan<int32_t>(s, sh, tot);
#pragma unroll
    for (int i = 0; i < kOrderPer; ++i) {
      cnt[tid * kOrderPer + i] = run;
      run += v[i];
    }
    __syncthreads();
    for (int32_t r = r_lo; r < r_hi; ++r) {
      const int32_t a = row_ptr[r], e = row_ptr[r + 1];
      for (int32_t q = a + tid; q < e; q += kOrderThreads) {
        const int32_t c = col_idx[q] - w0;
        if (c >= 0 && c < kOrderWin) order[base + cnt[c]++] = q;
      }
      __syncthreads();
    }
    base += tot;
  }
}

// ------------------------------------------------------------------ groups and panels
// Group cost w_g = blocks + rows of the group.
__global__ void k_group_cost(const int32_t* __restrict__ row_ptr, int32_t G, int32_t GR, int32_t mb,
                             int64_t* __restrict__ cost) {
  const int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const int32_t lo = g * GR, hi = min(mb, lo + GR);
  cost[g] = (int64_t)(row_ptr[hi] - row_ptr[lo]) + (hi - lo);
}

// In-place exclusive scan of G int64 costs into C[0..G] (C[G] = total); one block.
__global__ void k_cost_scan(int64_t* __restrict__ C, int32_t G) {
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
__global__ void k_panels(const int64_t* __restrict__ C, int32_t G, int32_t P, int32_t* __restrict__ panel_ptr) {
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

spmm_status_t build_static_plan(const uint8_t* mask_dev, int32_t mb, int32_t kb, const Geometry& geo,
                                PlanBuffers& pb, hipStream_t s) {
  int32_t* row_cnt = pb.scratch;        // [mb]
  int32_t* partials = pb.scratch + mb;  // scan partials
  const int rows_per_block = 4;
  dim3 grid((unsigned)ceil_div(mb, rows_per_block)), block(64 * rows_per_block);
  hipLaunchKernelGGL(k_static_count, grid, block, 0, s, mask_dev, mb, kb, row_cnt);
  spmm_status_t st = exscan_i32(row_cnt, pb.row_ptr, mb, partials, nullptr, s);
  if (st != SPMM_OK) return st;
  hipLaunchKernelGGL(k_static_fill, grid, block, 0, s, mask_dev, mb, kb, pb.row_ptr, pb.col_idx);
  const int32_t G = geo.num_groups;
  hipLaunchKernelGGL(k_group_order, dim3((unsigned)G), dim3(kOrderThreads), 0, s, pb.row_ptr, pb.col_idx, mb, kb,
                     geo.group_rows, pb.order);
  hipLaunchKernelGGL(k_group_cost, dim3((unsigned)ceil_div(G, 256)), dim3(256), 0, s, pb.row_ptr, G, geo.group_rows,
                     mb, pb.cost_prefix);
  hipLaunchKernelGGL(k_cost_scan, dim3(1), dim3(kScanThreads), 0, s, pb.cost_prefix, G);
  hipLaunchKernelGGL(k_panels, dim3((unsigned)ceil_div(geo.num_panels + 1, 256)), dim3(256), 0, s, pb.cost_prefix, G,
                     geo.num_panels, pb.panel_ptr);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

}  // namespace spmm
