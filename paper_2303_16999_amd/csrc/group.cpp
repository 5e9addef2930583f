// Grouped launch (C ABI): many static products in one launch of the row-wise
// kernel, one workgroup per work unit of all problems.
//
// Up to group_inline_max() problems travel in the kernel arguments: the call
// builds the table on the host and launches on it directly, or replays a
// captured one-node graph after updating that node's arguments and grid.
// Larger groups write the table into
// a pinned staging slot, copy it to the device and launch on it; the slots
// form a ring of kSlots, each reused only after the launch that read it has
// completed (an event per slot).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"

using namespace spmm;

namespace {
constexpr int kSlots = 4;
}

struct spmm_group_s {
  int32_t max_problems = 0;
  int device = 0;
  size_t desc_bytes = 0;
  size_t table_bytes = 0;
  uint8_t* host[kSlots] = {};  // pinned staging
  uint8_t* dev[kSlots] = {};
  hipEvent_t done[kSlots] = {};
  bool pending[kSlots] = {};
  int slot = 0;
  std::vector<uint8_t> args;    // argument-form table
  hipStream_t capture = nullptr;  // private stream used only to capture graphs
  struct Graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t node = nullptr;
  };
  std::map<std::tuple<int, int, int, bool>, Graph> graphs;  // (x, y, b, split rows)
  // piece workspace of the group's calls: each problem whose plan cuts long
  // rows into pieces takes its own range, so a plan may appear several times
  float* part = nullptr;
  int64_t part_cap = 0;  // bytes
  std::vector<std::pair<RunArgs, int32_t>> fixups;  // (problem, tile width) of a call's cut rows
};

static void destroy_group(spmm_group_s* g) {
  for (auto& kv : g->graphs) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
  }
  for (int s = 0; s < kSlots; ++s) {
    if (g->pending[s] && g->done[s]) (void)hipEventSynchronize(g->done[s]);
    if (g->done[s]) (void)hipEventDestroy(g->done[s]);
    if (g->host[s]) (void)hipHostFree(g->host[s]);
    if (g->dev[s]) (void)hipFree(g->dev[s]);
  }
  if (g->capture) (void)hipStreamDestroy(g->capture);
  if (g->part) (void)hipFree(g->part);
  delete g;
}

// The argument form launches directly unless SPMM_GROUP_GRAPH=1 asks for the
// graph replay: a replay (node update + hipGraphLaunch) measured about 5 us
// slower per call than the direct launch of the same kernel and arguments.
static bool use_graphs() {
  const char* e = getenv("SPMM_GROUP_GRAPH");
  return e && std::string(e) == "1";
}

// SPMM_GROUP_PERSIST=1 runs the persistent form (a CU-sized grid walking the
// units on a static per-XCD schedule), 0 the launch with one workgroup per
// unit.
static bool use_persist() {
  const char* e = getenv("SPMM_GROUP_PERSIST");
  return e && std::string(e) == "1";
}

// The captured one-node graph of the argument form for a dtype class: captured
// once with the current arguments, then only its node parameters change.
static spmm_status_t graph_for(spmm_group_s* g, spmm_dtype_t x, spmm_dtype_t y, int32_t b, unsigned lds,
                               int32_t total, spmm_group_s::Graph** out) {
  const auto key = std::make_tuple((int)x, (int)y, (int)b, lds > 0);
  auto it = g->graphs.find(key);
  if (it != g->graphs.end()) {
    *out = &it->second;
    return SPMM_OK;
  }
  spmm_group_s::Graph gr;
  SPMM_HIP(hipStreamBeginCapture(g->capture, hipStreamCaptureModeThreadLocal));
  spmm_status_t st = launch_spmm_row_grouped_args(x, y, b, g->args.data(), total, lds, g->capture);
  hipError_t e = hipStreamEndCapture(g->capture, &gr.graph);
  if (st != SPMM_OK) {
    if (gr.graph) (void)hipGraphDestroy(gr.graph);
    return st;
  }
  if (e != hipSuccess) return fail_hip(e, "hipStreamEndCapture");
  size_t nodes = 1;
  e = hipGraphGetNodes(gr.graph, &gr.node, &nodes);
  if (e == hipSuccess && nodes != 1) e = hipErrorInvalidValue;
  if (e == hipSuccess) e = hipGraphInstantiate(&gr.exec, gr.graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(gr.graph);
    return fail_hip(e, "grouped graph");
  }
  *out = &(g->graphs[key] = gr);
  return SPMM_OK;
}

// Grows the group's piece workspace to part_bytes, after the device has
// finished the launches that may still use the old one. False when it cannot
// grow now (the stream is being captured, or allocation failed): the call
// then splits long rows over one workgroup each.
static bool group_piece_workspace(spmm_group_s* g, int64_t part_bytes, hipStream_t s) {
  if (part_bytes <= g->part_cap) return true;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return false;
  if (g->part) {
    if (hipDeviceSynchronize() != hipSuccess) return false;
    (void)hipFree(g->part);
    g->part = nullptr;
    g->part_cap = 0;
  }
  const int64_t pb = std::max(part_bytes, 2 * g->part_cap);
  if (hipMalloc((void**)&g->part, (size_t)pb) != hipSuccess) {
    g->part = nullptr;
    return false;
  }
  g->part_cap = pb;
  return true;
}

// Partial bytes of one problem with pieces at tile width ns, 256-aligned.
static int64_t piece_bytes(const spmm_plan_s* p, int64_t n, int32_t ns) {
  return ((int64_t)p->num_slots * ceil_div(n, 16 * ns) * ns * 256 * 4 + 255) & ~(int64_t)255;
}

// The argument-form launch as a replay of the captured one-node graph, its
// node's arguments and grid updated.
static spmm_status_t replay_graph(spmm_group_s* g, const spmm_plan_s* p0, unsigned lds, int32_t total,
                                  hipStream_t strm) {
  spmm_group_s::Graph* gr = nullptr;
  spmm_status_t st = graph_for(g, p0->x, p0->y, p0->b, lds, total, &gr);
  if (st != SPMM_OK) return st;
  void* params[1] = {g->args.data()};
  hipKernelNodeParams kp{};
  kp.func = const_cast<void*>(row_grouped_args_kernel(p0->x, p0->y, p0->b, lds > 0));
  kp.gridDim = dim3((unsigned)total);
  kp.blockDim = dim3(256);
  kp.sharedMemBytes = lds;
  kp.kernelParams = params;
  kp.extra = nullptr;
  SPMM_HIP(hipGraphExecKernelNodeSetParams(gr->exec, gr->node, &kp));
  SPMM_HIP(hipGraphLaunch(gr->exec, strm));
  return SPMM_OK;
}

// The fixup launches of the call's problems with cut rows, after its launch.
static spmm_status_t run_fixups(spmm_group_s* g, hipStream_t strm) {
  for (const auto& f : g->fixups) {
    const spmm_status_t st = launch_group_fixup(f.first, f.second, strm);
    if (st != SPMM_OK) return st;
  }
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
  g->table_bytes = (size_t)max_problems * g->desc_bytes;
  spmm_status_t st = SPMM_OK;
  try {
    g->args.assign(group_args_bytes(), 0);
  } catch (...) {
    st = fail(SPMM_ERR_OOM, "host allocation failed");
  }
  hipError_t e = hipGetDevice(&g->device);
  if (st == SPMM_OK && e != hipSuccess) st = fail_hip(e, "hipGetDevice");
  const bool table = max_problems > group_inline_max();
  for (int s = 0; s < kSlots && st == SPMM_OK && table; ++s) {
    if ((e = hipHostMalloc((void**)&g->host[s], g->table_bytes, hipHostMallocDefault)) != hipSuccess)
      st = fail_hip(e, "hipHostMalloc");
    else if ((e = hipMalloc((void**)&g->dev[s], g->table_bytes)) != hipSuccess)
      st = fail_hip(e, "hipMalloc");
    else if ((e = hipEventCreateWithFlags(&g->done[s], hipEventDisableTiming)) != hipSuccess)
      st = fail_hip(e, "hipEventCreate");
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
  if (!plan_uses_row_kernel(p0) || p0->w == SPMM_FP8_E4M3 || p0->b > 32)
    return fail(SPMM_ERR_UNSUPPORTED, "grouped launch needs b = 16 or 32 with 16-bit W and X");
  int32_t used = 0;
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
    ++used;
  }
  if (used == 0) return SPMM_OK;
  const bool inline_table = used <= group_inline_max();
  const int s = g->slot;
  if (!inline_table && g->pending[s]) {
    SPMM_HIP(hipEventSynchronize(g->done[s]));
    g->pending[s] = false;
  }
  hipStream_t strm = (hipStream_t)stream;
  // the piece workspace the call needs (problems whose plan cuts long rows)
  int64_t need_part = 0;
  for (int32_t i = 0; i < count; ++i) {
    const spmm_plan_s* p = plans[i];
    if (n[i] == 0 || !p->num_slots) continue;
    const int32_t var = plan_variant(p, n[i]);
    int32_t ns = variant_ns(var);
    if (ns != 2 && ns != 4 && ns != 8) ns = default_ns(n[i]);
    if (!plan_pieces(p, n[i], ns, plan_split_all(p, n[i], ns, var))) continue;
    need_part += piece_bytes(p, n[i], ns);
  }
  const bool pieces = need_part > 0 && group_piece_workspace(g, need_part, strm);
  int64_t part_off = 0;
  g->fixups.clear();
  // descriptors, in call order, with the prefix of their work units
  int64_t total = 0, real_units = 0;
  int32_t k = 0;
  bool any_heavy = false;
  for (int32_t i = 0; i < count; ++i) {
    if (n[i] == 0) continue;
    const spmm_plan_s* p = plans[i];
    // the tuned variant if any, else the rule on n
    const int32_t var = plan_variant(p, n[i]);
    int32_t ns = variant_ns(var);
    if (ns != 2 && ns != 4 && ns != 8) ns = default_ns(n[i]);
    RunArgs a{};
    a.plan.m = (int32_t)p->m;
    a.plan.k = (int32_t)p->k;
    a.plan.b = p->b;
    a.plan.mb = p->mb;
    a.plan.kb = p->kb;
    a.W = p->values;
    a.scales = nullptr;
    a.X = X[i];
    a.Y = Y[i];
    a.ldx = ldx[i];
    a.ldy = ldy[i];
    a.n = (int32_t)n[i];
    a.relu = relu && relu[i];
    a.wt = p->w;
    a.xt = p->x;
    a.yt = p->y;
    a.ns = ns;
    a.num_heavy = p->num_heavy;
    a.light_rows = p->light_rows;
    a.num_light = p->mb - p->num_heavy;
    a.heavy_rows = p->heavy_rows;
    a.split_all = plan_split_all(p, n[i], ns, var);  // as the problem's own spmm_run_static would
    if (pieces && plan_pieces(p, n[i], ns, a.split_all)) {  // long rows cut into pieces, as in a single run
      a.num_heavy = a.split_all ? p->num_pieces_all : p->num_pieces;
      a.heavy_rows = a.split_all ? p->pieces_all : p->pieces;
      a.part = (float*)((uint8_t*)g->part + part_off);
      a.cut_rows = p->cut_rows;
      a.num_cut = p->num_cut;
      part_off += piece_bytes(p, n[i], ns);
      g->fixups.emplace_back(a, ns);
    }
    any_heavy = any_heavy || p->num_heavy > 0 || a.split_all;
    void* dst = inline_table ? group_args_problem(g->args.data(), k) : (void*)(g->host[s] + (size_t)k * g->desc_bytes);
    const int64_t units =
        a.split_all ? group_problem_units(0, n[i], ns, a.part ? a.num_heavy : p->mb, false)
                    : group_problem_units(a.light_rows ? a.num_light : p->mb, n[i], ns, a.num_heavy,
                                          a.part != nullptr && (a.light_rows ? a.num_light : p->mb) > 0);
    if (units >= (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "too many work units in one group");
    fill_row_problem(dst, a, p->pb.row_ptr, p->pb.col_idx, (int32_t)total, (int32_t)units);
    real_units += units;
    total += (units + 7) & ~(int64_t)7;  // each problem's range starts at a multiple of 8
    if (total >= (int64_t)INT32_MAX) return fail(SPMM_ERR_UNSUPPORTED, "too many work units in one group");
    ++k;
  }
  const unsigned lds = any_heavy ? group_split_lds(p0->b) : 0u;
  const bool persist = use_persist();
  const int32_t grid = group_persist_grid((int32_t)real_units, p0->b == 16 ? 4 : 3);
  if (inline_table) {
    group_args_header(g->args.data(), used, (int32_t)total);
    if (persist)
      st = launch_spmm_row_grouped_persist(p0->x, p0->y, p0->b, g->args.data(), nullptr, used, grid, lds, strm);
    else if (!use_graphs())
      st = launch_spmm_row_grouped_args(p0->x, p0->y, p0->b, g->args.data(), (int32_t)total, lds, strm);
    else
      st = replay_graph(g, p0, lds, (int32_t)total, strm);
    return st == SPMM_OK ? run_fixups(g, strm) : st;
  }
  SPMM_HIP(hipMemcpyAsync(g->dev[s], g->host[s], (size_t)used * g->desc_bytes, hipMemcpyHostToDevice, strm));
  st = persist ? launch_spmm_row_grouped_persist(p0->x, p0->y, p0->b, nullptr, g->dev[s], used, grid, lds, strm)
               : launch_spmm_row_grouped(p0->x, p0->y, p0->b, g->dev[s], used, (int32_t)total, lds, strm);
  if (st != SPMM_OK) return st;
  SPMM_HIP(hipEventRecord(g->done[s], strm));
  g->pending[s] = true;
  g->slot = (s + 1) % kSlots;
  return run_fixups(g, strm);
}


spmm_status_t spmm_group_destroy(spmm_group_t g) {
  clear_error();
  if (!g) return SPMM_OK;
  destroy_group(g);
  return SPMM_OK;
}

}  // extern "C"
