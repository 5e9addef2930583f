// Grouped persistent launch (C ABI): many static products in one launch of
// the row-wise kernel. The problem table is double-buffered: slot s has a
// pinned host staging copy, a device copy and an event recorded after the
// kernel that read it; a call fills the free slot, then replays the captured
// graph [copy host table s -> device table s; persistent kernel on table s].
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>

#include "internal.h"

using namespace spmm;

namespace {
constexpr size_t kHeaderBytes = 256;  // {count, total units}, padded so descriptors stay aligned
}

struct spmm_group_s {
  int32_t max_problems = 0;
  int device = 0;
  size_t desc_bytes = 0;
  size_t table_bytes = 0;
  uint8_t* host[2] = {nullptr, nullptr};  // pinned staging
  uint8_t* dev[2] = {nullptr, nullptr};
  hipEvent_t done[2] = {nullptr, nullptr};
  bool pending[2] = {false, false};
  int slot = 0;
  hipStream_t capture = nullptr;  // private stream used only to capture graphs
  std::map<std::tuple<int, int, int, int>, hipGraphExec_t> graphs;  // (x, y, b, slot)
  std::map<std::tuple<int, int, int>, int32_t> grids;               // (x, y, b)
};

static void destroy_group(spmm_group_s* g) {
  for (auto& kv : g->graphs) (void)hipGraphExecDestroy(kv.second);
  for (int s = 0; s < 2; ++s) {
    if (g->pending[s] && g->done[s]) (void)hipEventSynchronize(g->done[s]);
    if (g->done[s]) (void)hipEventDestroy(g->done[s]);
    if (g->host[s]) (void)hipHostFree(g->host[s]);
    if (g->dev[s]) (void)hipFree(g->dev[s]);
  }
  if (g->capture) (void)hipStreamDestroy(g->capture);
  delete g;
}

static bool use_graphs() {
  const char* e = getenv("SPMM_GROUP_GRAPH");
  return !(e && std::string(e) == "0");
}

// Enqueues [table copy, grouped kernel] for slot s directly on `stream`.
static spmm_status_t enqueue_direct(spmm_group_s* g, int s, spmm_dtype_t x, spmm_dtype_t y, int32_t b, int32_t grid,
                                    hipStream_t stream) {
  SPMM_HIP(hipMemcpyAsync(g->dev[s], g->host[s], g->table_bytes, hipMemcpyHostToDevice, stream));
  return launch_spmm_row_grouped(x, y, b, g->dev[s] + kHeaderBytes, (const int32_t*)g->dev[s], grid, stream);
}

static spmm_status_t graph_for(spmm_group_s* g, int s, spmm_dtype_t x, spmm_dtype_t y, int32_t b, int32_t grid,
                               hipGraphExec_t* out) {
  const auto key = std::make_tuple((int)x, (int)y, (int)b, s);
  auto it = g->graphs.find(key);
  if (it != g->graphs.end()) {
    *out = it->second;
    return SPMM_OK;
  }
  SPMM_HIP(hipStreamBeginCapture(g->capture, hipStreamCaptureModeThreadLocal));
  spmm_status_t st = enqueue_direct(g, s, x, y, b, grid, g->capture);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(g->capture, &graph);
  if (st != SPMM_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return fail_hip(e, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail_hip(e, "hipGraphInstantiate");
  g->graphs[key] = exec;
  *out = exec;
  return SPMM_OK;
}

extern "C" {

spmm_status_t spmm_group_create(int32_t max_problems, spmm_group_t* out) {
  clear_error();
  if (!out) return fail(SPMM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (max_problems < 1 || max_problems > 65536) return fail(SPMM_ERR_INVALID_ARG, "max_problems must be in [1, 65536]");
  spmm_group_s* g = new (std::nothrow) spmm_group_s;
  if (!g) return fail(SPMM_ERR_OOM, "host allocation failed");
  g->max_problems = max_problems;
  g->desc_bytes = row_problem_size();
  g->table_bytes = kHeaderBytes + (size_t)max_problems * g->desc_bytes;
  spmm_status_t st = SPMM_OK;
  hipError_t e = hipGetDevice(&g->device);
  if (e != hipSuccess) st = fail_hip(e, "hipGetDevice");
  for (int s = 0; s < 2 && st == SPMM_OK; ++s) {
    if ((e = hipHostMalloc((void**)&g->host[s], g->table_bytes, hipHostMallocDefault)) != hipSuccess)
      st = fail_hip(e, "hipHostMalloc");
    else if ((e = hipMalloc((void**)&g->dev[s], g->table_bytes)) != hipSuccess)
      st = fail_hip(e, "hipMalloc");
    else if ((e = hipEventCreateWithFlags(&g->done[s], hipEventDisableTiming)) != hipSuccess)
      st = fail_hip(e, "hipEventCreate");
    if (st == SPMM_OK) std::memset(g->host[s], 0, g->table_bytes);
  }
  if (st == SPMM_OK && (e = hipStreamCreateWithFlags(&g->capture, hipStreamNonBlocking)) != hipSuccess)
    st = fail_hip(e, "hipStreamCreate");
  if (st != SPMM_OK) {
    destroy_group(g);
    return st;
  }
  *out = g;
  return SPMM_OK;
}

spmm_status_t spmm_group_run(spmm_group_t g, int32_t count, const spmm_plan_t* plans, const int64_t* n,
                             const void* const* X, const int64_t* ldx, void* const* Y, const int64_t* ldy,
                             const uint8_t* relu, void* stream) {
  clear_error();
  if (!g) return fail(SPMM_ERR_INVALID_ARG, "group handle is NULL");
  if (count < 0 || count > g->max_problems) return fail(SPMM_ERR_INVALID_ARG, "count outside [0, max_problems]");
  if (count == 0) return SPMM_OK;
  if (!plans || !n || !X || !ldx || !Y || !ldy) return fail(SPMM_ERR_INVALID_ARG, "NULL array argument");
  spmm_status_t st = check_device(g->device);
  if (st != SPMM_OK) return st;
  const spmm_plan_s* p0 = plans[0];
  if (!p0) return fail(SPMM_ERR_INVALID_ARG, "plan 0 is NULL");
  if (!plan_uses_row_kernel(p0) || p0->w == SPMM_FP8_E4M3)
    return fail(SPMM_ERR_UNSUPPORTED, "grouped launch needs b = 16 or 32 with 16-bit W and X");
  for (int32_t i = 0; i < count; ++i) {
    const spmm_plan_s* p = plans[i];
    if (!p) return fail(SPMM_ERR_INVALID_ARG, "a plan is NULL");
    if (p->b != p0->b || p->w != p0->w || p->x != p0->x || p->y != p0->y)
      return fail(SPMM_ERR_INVALID_ARG, "plans of one group must share block size and dtypes");
    if (p->device != g->device) return fail(SPMM_ERR_INVALID_ARG, "plan lives on another device");
    if (!p->has_values) return fail(SPMM_ERR_INVALID_ARG, "values were not set on a plan");
    if (n[i] < 0 || n[i] > INT32_MAX / 2) return fail(SPMM_ERR_INVALID_ARG, "n outside [0, 2^30]");
    if (n[i] == 0) continue;
    if ((st = check_dense(X[i], ldx[i], n[i], dtype_bytes(p->x), "X")) != SPMM_OK) return st;
    if ((st = check_dense(Y[i], ldy[i], n[i], dtype_bytes(p->y), "Y")) != SPMM_OK) return st;
    if (p->k * ldx[i] * 2 >= (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "X larger than 2 GiB");
  }
  const int s = g->slot;
  if (g->pending[s]) {
    SPMM_HIP(hipEventSynchronize(g->done[s]));
    g->pending[s] = false;
  }
  uint8_t* tab = g->host[s];
  int64_t total = 0;
  int32_t used = 0;
  for (int32_t i = 0; i < count; ++i) {
    if (n[i] == 0) continue;
    const spmm_plan_s* p = plans[i];
    // the tuned variant if any, else the widest tile n fills at least half of
    // (the group as a whole fills the chip, so no narrowing for occupancy)
    int32_t ns = plan_variant(p, n[i]);
    if (ns != 2 && ns != 4 && ns != 8) ns = n[i] > 64 ? 8 : (n[i] > 32 ? 4 : 2);
    RunArgs a{};
    a.plan.m = (int32_t)p->m;
    a.plan.k = (int32_t)p->k;
    a.plan.b = p->b;
    a.plan.mb = p->mb;
    a.plan.kb = p->kb;
    a.W = p->values_csr;
    a.scales = nullptr;
    a.X = X[i];
    a.Y = Y[i];
    a.ldx = ldx[i];
    a.ldy = ldy[i];
    a.n = (int32_t)n[i];
    a.relu = relu && relu[i];
    a.ns = ns;
    fill_row_problem(tab + kHeaderBytes + (size_t)used * g->desc_bytes, a, p->pb.row_ptr, p->pb.col_idx,
                     (int32_t)total);
    total += ceil_div(p->mb, 4) * ceil_div(n[i], 16 * ns);
    if (total >= (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "too many work units in one group");
    ++used;
  }
  if (used == 0) return SPMM_OK;
  ((int32_t*)tab)[0] = used;
  ((int32_t*)tab)[1] = (int32_t)total;
  const auto gk = std::make_tuple((int)p0->x, (int)p0->y, (int)p0->b);
  auto git = g->grids.find(gk);
  int32_t grid;
  if (git == g->grids.end()) {
    grid = row_grouped_grid(p0->x, p0->y, p0->b);
    g->grids[gk] = grid;
  } else {
    grid = git->second;
  }
  hipStream_t strm = (hipStream_t)stream;
  if (use_graphs()) {
    hipGraphExec_t exec = nullptr;
    if ((st = graph_for(g, s, p0->x, p0->y, p0->b, grid, &exec)) != SPMM_OK) return st;
    SPMM_HIP(hipGraphLaunch(exec, strm));
  } else {
    if ((st = enqueue_direct(g, s, p0->x, p0->y, p0->b, grid, strm)) != SPMM_OK) return st;
  }
  SPMM_HIP(hipEventRecord(g->done[s], strm));
  g->pending[s] = true;
  g->slot = s ^ 1;
  return SPMM_OK;
}

spmm_status_t spmm_group_destroy(spmm_group_t g) {
  clear_error();
  if (!g) return SPMM_OK;
  destroy_group(g);
  return SPMM_OK;
}

}  // extern "C"
