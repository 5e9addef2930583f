// Host side of the C ABI: argument validation, handles, device buffers and
// kernel dispatch. No arithmetic of the SpMM happens here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"

namespace spmm {

static thread_local std::string g_last_error;

spmm_status_t fail(spmm_status_t st, const std::string& msg) {
  g_last_error = msg;
  return st;
}
spmm_status_t fail_hip(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? SPMM_ERR_OOM : SPMM_ERR_HIP;
}
void clear_error() { g_last_error.clear(); }

int dtype_bytes(spmm_dtype_t t) {
  switch (t) {
    case SPMM_F32: return 4;
    case SPMM_F16: return 2;
    case SPMM_BF16: return 2;
    case SPMM_FP8_E4M3: return 1;
  }
  return 0;
}

bool dtype_triple_supported(spmm_dtype_t w, spmm_dtype_t x, spmm_dtype_t y) {
  if (w == SPMM_F32) return x == SPMM_F32 && y == SPMM_F32;
  if (w == SPMM_F16) return x == SPMM_F16 && (y == SPMM_F16 || y == SPMM_F32);
  if (w == SPMM_BF16) return x == SPMM_BF16 && (y == SPMM_BF16 || y == SPMM_F32);
  if (w == SPMM_FP8_E4M3) return (x == SPMM_F16 || x == SPMM_BF16) && (y == x || y == SPMM_F32);
  return false;
}

int device_cu_count() {
  static int cached[64] = {};
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess) return cus;
  if (dev >= 0 && dev < 64 && cached[dev] > 0) return cached[dev];
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  if (dev >= 0 && dev < 64) cached[dev] = cus;
  return cus;
}

static bool valid_block(int32_t b) { return b == 1 || b == 4 || b == 8 || b == 16 || b == 32; }
// Static plans also take b = 64 (4 x 4 MFMA tiles of 16, 16-bit X).
static bool valid_static_block(int32_t b) { return valid_block(b) || b == 64; }

Geometry choose_geometry(int64_t m, int64_t k, int32_t b, int64_t nnz_hint, int64_t n_hint,
                         const spmm_plan_opts* opts, int num_cus, spmm_dtype_t x) {
  (void)k;
  (void)nnz_hint;
  (void)x;
  Geometry g{};
  const int64_t mb = ceil_div(m, b);
  if (n_hint <= 0) n_hint = 1024;
  // row groups of the plan: large where groups x n-tiles still gives every CU
  // two units, else small
  int32_t big = 0, small = 0, ntile = 128;
  if (b >= 16) { big = b == 16 ? 32 : (b == 32 ? 16 : 8); small = b == 16 ? 8 : (b == 32 ? 4 : 2); }
  else { big = 64; small = 16; ntile = 64; }
  int32_t gr = big;
  if (ceil_div(mb, big) * ceil_div(n_hint, ntile) < 2 * (int64_t)num_cus) gr = small;
  if (const char* e = getenv("SPMM_GROUP_ROWS")) {  // tuning override
    const int v = atoi(e);
    if (v > 0) gr = v;
  }
  if (opts && opts->group_rows > 0) gr = opts->group_rows;
  g.group_rows = gr;
  g.num_groups = (int32_t)ceil_div(mb, gr);
  g.num_panels = (opts && opts->num_panels > 0) ? std::min<int32_t>(opts->num_panels, g.num_groups) : g.num_groups;
  if (g.num_panels < 1) g.num_panels = 1;
  return g;
}

// Column tiles of 16 per wave for the row-wise kernel: the widest tile that
// the n columns fill at least half of. (Measured on MI355X, the widest tile is
// also fastest when a launch has only one workgroup per CU: narrower tiles
// re-read the weights more often than the extra occupancy pays back.)
int32_t default_ns(int64_t n) { return n > 64 ? 8 : (n > 32 ? 4 : 2); }

// Dynamic encoders, in order of preference where they apply: the row-range
// encoder (one launch, many workgroups), the one-workgroup encoder, the
// multi-kernel one. Both single-launch encoders need b to divide k (values are
// read in place). SPMM_DYN_BUILDER=rows|one|multi asks for one of them (for
// comparisons; a builder that does not apply falls through to the next).
enum DynBuilder { kBuilderNone = 0, kBuilderRows = 1, kBuilderOne = 2, kBuilderMulti = 3 };
static int requested_builder() {
  const char* e = getenv("SPMM_DYN_BUILDER");
  if (!e) return kBuilderNone;
  const std::string v(e);
  if (v == "rows") return kBuilderRows;
  if (v == "one") return kBuilderOne;
  if (v == "multi") return kBuilderMulti;
  return kBuilderNone;
}

static void free_plan_buffers(PlanBuffers& pb) {
  int32_t* ptrs[] = {pb.panel_ptr, pb.row_ptr, pb.col_idx, pb.order, pb.csr_src, pb.tmp_col, pb.tmp_src,
                     pb.scratch, pb.hist};
  for (int32_t* p : ptrs)
    if (p) (void)hipFree(p);
  if (pb.cost_prefix) (void)hipFree(pb.cost_prefix);
  pb = PlanBuffers{};
}

template <typename T>
static spmm_status_t dev_alloc(T** p, int64_t count) {
  *p = nullptr;
  if (count <= 0) count = 1;
  hipError_t e = hipMalloc((void**)p, (size_t)count * sizeof(T));
  if (e != hipSuccess) return fail_hip(e, "hipMalloc");
  return SPMM_OK;
}

static spmm_status_t alloc_plan_buffers(PlanBuffers& pb, const Geometry& geo, int32_t mb, int64_t nnz, bool dynamic) {
  spmm_status_t st;
  const int64_t scan_parts = ceil_div(std::max<int64_t>(mb, 1), 1024) + 16;
  pb.scratch_ints = (dynamic ? 2 * (int64_t)mb : (int64_t)mb) + scan_parts + 16;
  if ((st = dev_alloc(&pb.panel_ptr, (int64_t)geo.num_panels + 1)) != SPMM_OK) return st;
  if ((st = dev_alloc(&pb.row_ptr, (int64_t)mb + 1)) != SPMM_OK) return st;
  if ((st = dev_alloc(&pb.col_idx, nnz)) != SPMM_OK) return st;
  if (!dynamic && (st = dev_alloc(&pb.order, nnz)) != SPMM_OK) return st;
  if (dynamic && (st = dev_alloc(&pb.csr_src, nnz)) != SPMM_OK) return st;
  if (dynamic && (st = dev_alloc(&pb.tmp_col, nnz)) != SPMM_OK) return st;
  if (dynamic && (st = dev_alloc(&pb.tmp_src, nnz)) != SPMM_OK) return st;
  if ((st = dev_alloc(&pb.scratch, pb.scratch_ints)) != SPMM_OK) return st;
  if ((st = dev_alloc(&pb.cost_prefix, (int64_t)geo.num_groups + 1)) != SPMM_OK) return st;
  if (dynamic && (pb.hist_wgs = dyn_hist_wgs(nnz, mb)) > 0 &&
      (st = dev_alloc(&pb.hist, (int64_t)pb.hist_wgs * mb)) != SPMM_OK)
    return st;
  return SPMM_OK;
}

static KernelPlan kernel_plan(int64_t m, int64_t k, int32_t b, int32_t mb, int32_t kb, const Geometry& geo,
                              const PlanBuffers& pb) {
  KernelPlan kp;
  kp.m = (int32_t)m;
  kp.k = (int32_t)k;
  kp.b = b;
  kp.mb = mb;
  kp.kb = kb;
  kp.group_rows = geo.group_rows;
  kp.num_groups = geo.num_groups;
  kp.num_panels = geo.num_panels;
  kp.panel_ptr = pb.panel_ptr;
  kp.order = pb.order;
  return kp;
}

spmm_status_t check_dense(const void* p, int64_t ld, int64_t n, int elem, const char* name) {
  if (!p) return fail(SPMM_ERR_INVALID_ARG, std::string(name) + " is NULL");
  if (ld < n) return fail(SPMM_ERR_INVALID_ARG, std::string("leading dimension of ") + name + " is smaller than n");
  if (((uintptr_t)p) % 16 != 0) return fail(SPMM_ERR_INVALID_ARG, std::string(name) + " is not 16-byte aligned");
  if ((ld * elem) % 16 != 0)
    return fail(SPMM_ERR_INVALID_ARG, std::string("leading dimension of ") + name + " is not a multiple of 16 bytes");
  return SPMM_OK;
}

spmm_status_t check_device(int device) {
  int cur = -1;
  SPMM_HIP(hipGetDevice(&cur));
  if (cur != device) return fail(SPMM_ERR_INVALID_ARG, "handle was created on another device");
  return SPMM_OK;
}


// ------------------------------------------------------------------ tile variants
int n_class(int64_t n) {
  int c = 0;
  while (c < 31 && ((int64_t)1 << c) < n) ++c;
  return c;
}

bool plan_uses_row_kernel(const spmm_plan_s* p) {
  return p->b >= 16 && (p->x == SPMM_F16 || p->x == SPMM_BF16);
}

bool valid_variant(int32_t b, int32_t v) {
  if (v == 0) return true;
  if (v < 0) return false;
  const int32_t ns = variant_ns(v), form = variant_form(v);
  if (form > 5 || (ns != 0 && ns != 2 && ns != 4 && ns != 8)) return false;
  if (form == 5 && b != 16) return false;
  return !(ns == 2 && b < 16);
}

// Process-wide autotuner table: (b, w, x, y, density class, n class) ->
// variant. With SPMM_AUTOTUNE_CACHE naming a file, the table starts from that
// file (if it was written for this device and HIP runtime) and every new
// entry rewrites it.
static std::mutex g_tune_mu;
static std::map<TuneKey, int32_t> g_tune;
static bool g_tune_loaded = false;

static const char* tune_cache_path() {
  const char* e = getenv("SPMM_AUTOTUNE_CACHE");
  return e && *e ? e : nullptr;
}

// (call with g_tune_mu held)
static void tune_table_load_once() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  if (const char* path = tune_cache_path()) (void)tune_cache_load(path, g_tune);
}

static TuneKey tune_key(const spmm_plan_s* p, int64_t n) {
  const double cells = (double)p->mb * (double)p->kb;
  const double d = cells > 0 ? (double)p->nnzb / cells : 0.0;
  const int dclass = d > 0 ? (int)std::lround(-std::log2(d)) : 64;
  return TuneKey(p->b, (int)p->w, (int)p->x, (int)p->y, dclass, n_class(n), p->dense_w ? 1 : 0);
}

static void tune_table_put(const spmm_plan_s* p, int64_t n, int32_t v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_table_load_once();
  g_tune[tune_key(p, n)] = v;
  if (const char* path = tune_cache_path()) (void)tune_cache_save(path, g_tune);
}

int32_t plan_variant(const spmm_plan_s* p, int64_t n) {
  if (p->variant_opt) return p->variant_opt;
  const int32_t t = p->tuned[n_class(n)];
  if (t) return t;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_table_load_once();
    auto it = g_tune.find(tune_key(p, n));
    if (it != g_tune.end()) return it->second;
  }
  return 0;
}

bool plan_split_all(const spmm_plan_s* p, int64_t n, int32_t ns, int32_t variant) {
  if (p->b != 16 || !plan_uses_row_kernel(p)) return false;
  const int32_t form = variant_form(variant);
  if (form && !getenv("SPMM_SPLIT_ALL")) return form == 4;
  return split_all_preferred(p->b, p->mb, n, ns, p->nnzb, device_cu_count());
}

static bool piece_workspace(const spmm_plan_s* cp, int64_t n, hipStream_t s);

// Whether a run of n columns at tile width ns cuts the plan's long rows into
// pieces (the plan must have some): where its split rows differ widely in
// length, or where they alone would give fewer than two workgroups per CU
// (a single long row is the worst case). Otherwise the four-wave split
// balances them, and pieces would only add their partial sums' traffic and
// the fixup launch. SPMM_PIECES=0 / 1 forces the choice.
bool plan_pieces(const spmm_plan_s* p, int64_t n, int32_t ns, bool split_all) {
  if (!p->num_slots) return false;
  if (const char* e = getenv("SPMM_PIECES")) return e[0] != '0';
  if (p->pieces_spread) return true;
  const int64_t units = (int64_t)(split_all ? p->mb : p->num_heavy) * ceil_div(n, 16 * ns);
  return units < 2 * (int64_t)device_cu_count();
}

spmm_status_t run_plan(const spmm_plan_s* p, int64_t n, const void* X, int64_t ldx, void* Y, int64_t ldy,
                       int32_t variant, bool relu, hipStream_t stream) {
  RunArgs a{};
  a.plan = kernel_plan(p->m, p->k, p->b, p->mb, p->kb, p->geo, p->pb);
  a.W = p->values;
  a.scales = p->scales;
  a.X = X;
  a.Y = Y;
  a.ldx = ldx;
  a.ldy = ldy;
  a.n = (int32_t)n;
  a.wt = p->w;
  a.xt = p->x;
  a.yt = p->y;
  a.status = nullptr;
  a.nnz = p->nnzb;
  a.relu = relu;
  // a variant's kernel form applies where the plan has that form, unless the
  // environment forces one (SPMM_SMALL_LDS, SPMM_ROW_PP)
  const int32_t form = variant_form(variant);
  // the dense copy: when asked for, or by the rule where the model favours it
  // (never with a fused ReLU)
  if (p->dense_w && !relu && (form == 3 || (form == 0 && p->predicted_speedup < 1.0)))
    return run_dense(p, n, X, ldx, Y, ldy, stream);
  if (p->b < 16) {
    bool lds = small_lds_preferred(p->b, p->w, p->x, p->nnzb, p->mb, p->kb, n);
    if (form && small_lds_eligible(p->b, p->w, p->x) && !getenv("SPMM_SMALL_LDS")) lds = form == 2;
    if (lds)
      return launch_spmm_small_lds(a, p->pb.row_ptr, p->pb.col_idx,
                                   small_lds_rows_per_wave(p->b, p->mb, n, device_cu_count()), stream);
    a.ns = variant_ns(variant);  // 0: the kernel's rule on n
    return launch_spmm_small(a, p->pb.row_ptr, p->pb.col_idx, stream);
  }
  if (plan_uses_row_kernel(p)) {
    a.ns = variant_ns(variant) ? variant_ns(variant) : default_ns(n);
    a.num_heavy = p->num_heavy;
    a.light_rows = p->light_rows;
    a.num_light = p->mb - p->num_heavy;
    a.heavy_rows = p->heavy_rows;
    a.split_all = plan_split_all(p, n, a.ns, variant);
    if (plan_pieces(p, n, a.ns, a.split_all) && piece_workspace(p, n, stream)) {
      a.num_heavy = a.split_all ? p->num_pieces_all : p->num_pieces;
      a.heavy_rows = a.split_all ? p->pieces_all : p->pieces;
      a.part = p->piece_part;
      a.cut_rows = p->cut_rows;
      a.num_cut = p->num_cut;
    }
    if (a.split_all) return launch_spmm_row(a, p->pb.row_ptr, p->pb.col_idx, stream);
    const bool pp_ok = p->w == p->x && p->num_heavy == 0 && p->b <= 32;
    bool pp = pp_ok && row_pp_preferred(p->b, p->mb, n, a.ns, p->nnzb, device_cu_count());
    if (form && pp_ok && !getenv("SPMM_ROW_PP")) pp = form == 2;
    if (pp) return launch_spmm_row_pp(a, p->pb.row_ptr, p->pb.col_idx, stream);
    return launch_spmm_row(a, p->pb.row_ptr, p->pb.col_idx, stream);
  }
  return launch_spmm_row_f32(a, p->pb.row_ptr, p->pb.col_idx, stream);
}

// The compute kernel of a dynamic call on its block-CSR (no split-row table):
// variant 0 takes the rules, else its tile width and kernel form (forms 1
// plain, 2 pipelined row kernel or LDS-staged b = 4 kernel, 4 every row split)
// where the call's kernel has them; SPMM_SMALL_LDS, SPMM_ROW_PP and
// SPMM_SPLIT_ALL still force their choice.
spmm_status_t run_dynamic_kernel(RunArgs& a, const int32_t* row_ptr, const int32_t* col_idx, hipStream_t s,
                                 int32_t variant) {
  const int32_t b = a.plan.b;
  const int32_t form = variant_form(variant);
  const int cus = device_cu_count();
  if (b < 16) {
    bool lds = small_lds_preferred(b, a.wt, a.xt, a.nnz, a.plan.mb, a.plan.kb, a.n);
    if (form && small_lds_eligible(b, a.wt, a.xt) && !getenv("SPMM_SMALL_LDS")) lds = form == 2;
    if (lds) return launch_spmm_small_lds(a, row_ptr, col_idx, small_lds_rows_per_wave(b, a.plan.mb, a.n, cus), s);
    a.ns = variant_ns(variant);
    return launch_spmm_small(a, row_ptr, col_idx, s);
  }
  a.ns = variant_ns(variant) ? variant_ns(variant) : default_ns(a.n);
  if (a.xt == SPMM_F32) return launch_spmm_row_f32(a, row_ptr, col_idx, s);
  bool split = split_all_preferred(b, a.plan.mb, a.n, a.ns, a.nnz, cus);
  if (form && b == 16 && !getenv("SPMM_SPLIT_ALL")) split = form == 4;
  if (split) {
    a.split_all = true;
    return launch_spmm_row(a, row_ptr, col_idx, s);
  }
  const bool pp_ok = a.wt == a.xt && b <= 32;
  bool pp = pp_ok && row_pp_preferred(b, a.plan.mb, a.n, a.ns, a.nnz, cus);
  if (form && pp_ok && !getenv("SPMM_ROW_PP")) pp = form == 2;
  if (pp) return launch_spmm_row_pp(a, row_ptr, col_idx, s);
  return launch_spmm_row(a, row_ptr, col_idx, s);
}

// A run with no fixed and no tuned variant for its n class tunes first
// (SPMM_AUTOTUNE=0 keeps the rule instead), except on a stream under capture.
static bool tune_on_first_run(hipStream_t s) {
  const char* e = getenv("SPMM_AUTOTUNE");
  if (e && e[0] == '0') return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return false;
  return cs == hipStreamCaptureStatusNone;
}


// Candidate variants of a dynamic call: the compute kernel's forms after the
// encoder, and the one-launch form where it fits.
static int dynamic_candidates(int32_t b, spmm_dtype_t w, spmm_dtype_t x, bool fused, int32_t (&c)[10]) {
  int k = 0;
  if (b >= 16 && (x == SPMM_F16 || x == SPMM_BF16)) {
    for (int32_t ns : {2, 4, 8}) c[k++] = make_variant(ns, 1);
    if (w == x && b <= 32)
      for (int32_t ns : {2, 4, 8}) c[k++] = make_variant(ns, 2);
    if (b == 16) c[k++] = make_variant(0, 4);
    if (fused)
      for (int32_t ns : {2, 4, 8}) c[k++] = make_variant(ns, 5);
  } else if (b < 16 && x != SPMM_F32) {
    c[k++] = make_variant(4, 1);
    c[k++] = make_variant(8, 1);
    if (small_lds_eligible(b, w, x)) c[k++] = make_variant(0, 2);
  }
  return k;
}

// Tiled SDDMM tasks (b = 16/32): the blocks of each tile of T x T blocks (T =
// sddmm_tiled_tile_blocks), listed by block row then column, in tasks of at
// most sddmm_tiled_task_blocks; tiles in (tile row, tile column) order.
static spmm_status_t build_sddmm_tiled(spmm_plan_s* p, const std::vector<int32_t>& rp) {
  if (p->b != 16 && p->b != 32) return SPMM_OK;
  const int64_t nnz = p->nnzb;
  if (nnz == 0) return SPMM_OK;
  std::vector<int32_t> ci((size_t)nnz);
  SPMM_HIP(hipMemcpy(ci.data(), p->pb.col_idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
  const int32_t T = sddmm_tiled_tile_blocks(p->b), cap = sddmm_tiled_task_blocks(p->b);
  const int32_t tcols = (int32_t)ceil_div(p->kb, T);
  std::vector<int32_t> ent, tasks;
  ent.reserve((size_t)nnz * 2);
  std::vector<std::vector<int32_t>> tile((size_t)tcols);  // CSR indices per tile column of one tile row
  for (int32_t tr = 0; tr * T < p->mb; ++tr) {
    for (auto& v : tile) v.clear();
    for (int32_t r = tr * T; r < std::min(p->mb, (tr + 1) * T); ++r)
      for (int32_t q = rp[r]; q < rp[r + 1]; ++q) tile[ci[q] / T].push_back(q);
    for (int32_t tc = 0; tc < tcols; ++tc) {
      const std::vector<int32_t>& v = tile[tc];
      for (size_t o = 0; o < v.size(); o += cap) {
        tasks.push_back(tr);
        tasks.push_back(tc);
        tasks.push_back((int32_t)(ent.size() / 2));
        tasks.push_back((int32_t)std::min<size_t>(cap, v.size() - o));
        for (size_t e = o; e < std::min(v.size(), o + cap); ++e) {
          const int32_t q = v[e];
          int32_t r = 0;  // block row of entry q: the row whose range holds it
          r = (int32_t)(std::upper_bound(rp.begin(), rp.end(), q) - rp.begin()) - 1;
          ent.push_back(q);
          ent.push_back(((r - tr * T) << 16) | (ci[q] - tc * T));
        }
      }
    }
  }
  p->sddmm_tiled_num = (int32_t)(tasks.size() / 4);
  spmm_status_t st = dev_alloc(&p->sddmm_tiled_tasks, (int64_t)tasks.size());
  if (st == SPMM_OK) st = dev_alloc(&p->sddmm_tiled_ent, (int64_t)ent.size());
  if (st != SPMM_OK) return st;
  SPMM_HIP(hipMemcpy(p->sddmm_tiled_tasks, tasks.data(), sizeof(int32_t) * tasks.size(), hipMemcpyHostToDevice));
  SPMM_HIP(hipMemcpy(p->sddmm_tiled_ent, ent.data(), sizeof(int32_t) * ent.size(), hipMemcpyHostToDevice));
  return SPMM_OK;
}

// SDDMM tasks of a plan: (block row, first entry) for every run of up to
// sddmm_task_blocks(b) consecutive blocks of one row.
static spmm_status_t build_sddmm_tasks(spmm_plan_s* p, const std::vector<int32_t>& rp) {
  const int32_t per = sddmm_task_blocks(p->b);
  std::vector<int32_t> tasks;
  for (int32_t r = 0; r < p->mb; ++r)
    for (int32_t q = rp[r]; q < rp[r + 1]; q += per) {
      tasks.push_back(r);
      tasks.push_back(q);
    }
  p->sddmm_num_tasks = (int32_t)(tasks.size() / 2);
  if (tasks.empty()) return SPMM_OK;
  spmm_status_t st = dev_alloc(&p->sddmm_tasks, (int64_t)tasks.size());
  if (st != SPMM_OK) return st;
  SPMM_HIP(hipMemcpy(p->sddmm_tasks, tasks.data(), sizeof(int32_t) * tasks.size(), hipMemcpyHostToDevice));
  return SPMM_OK;
}

// Long rows to split, and the order in which light units take the others.
// Rows with more than max(64, 2 x mean) blocks are split over a workgroup's
// four waves, and rows longer than max(256, 2 x that limit) blocks can also
// be cut into pieces of about that many blocks, one workgroup each (a fixup
// launch adds the pieces' partial sums in piece order; plan_pieces decides
// per run). Where some row is split, or the longest row holds more than
// twice the mean, the light units take the remaining rows longest first (a
// unit's waves then hold rows of about the same length, and the long ones
// start early), else in order. SPMM_SPLIT=0 turns all three off,
// SPMM_ROW_ORDER=0 the order; SPMM_SPLIT_BLOCKS sets the split limit,
// SPMM_PIECE_BLOCKS the piece length.
static spmm_status_t classify_heavy_rows(spmm_plan_s* p, const std::vector<int32_t>& rp) {
  const char* e = getenv("SPMM_SPLIT");
  if (e && std::string(e) == "0") return SPMM_OK;
  if (p->mb == 0 || p->nnzb == 0) return SPMM_OK;
  const int64_t mean = ceil_div(p->nnzb, p->mb);
  int64_t limit = std::max<int64_t>(64, 2 * mean);
  if (const char* sb = getenv("SPMM_SPLIT_BLOCKS")) limit = std::max<int64_t>(8, atoll(sb));
  std::vector<int32_t> heavy, light;
  int64_t longest = 0;
  for (int32_t r = 0; r < p->mb; ++r) {
    const int64_t len = rp[r + 1] - rp[r];
    longest = std::max(longest, len);
    if (len > limit) heavy.push_back(r);
    else light.push_back(r);
  }
  const char* o = getenv("SPMM_ROW_ORDER");
  const bool order = (o && o[0] == '2') || (!(o && o[0] == '0') && (!heavy.empty() || longest > 2 * mean));
  spmm_status_t st = SPMM_OK;
  if (!heavy.empty()) {
    if ((st = dev_alloc(&p->heavy_rows, (int64_t)heavy.size())) != SPMM_OK) return st;
    SPMM_HIP(hipMemcpy(p->heavy_rows, heavy.data(), sizeof(int32_t) * heavy.size(), hipMemcpyHostToDevice));
    p->num_heavy = (int32_t)heavy.size();
  }
  if (order || !heavy.empty()) {  // with split rows the list also leaves them out
    if (order)
      std::stable_sort(light.begin(), light.end(),
                       [&](int32_t a, int32_t b) { return rp[a + 1] - rp[a] > rp[b + 1] - rp[b]; });
    if ((st = dev_alloc(&p->light_rows, (int64_t)light.size())) != SPMM_OK) return st;
    if (!light.empty())
      SPMM_HIP(hipMemcpy(p->light_rows, light.data(), sizeof(int32_t) * light.size(), hipMemcpyHostToDevice));
  }
  if (heavy.empty()) return SPMM_OK;
  int64_t piece = std::max<int64_t>(256, 2 * limit);
  if (const char* pb = getenv("SPMM_PIECE_BLOCKS")) piece = std::max<int64_t>(16, atoll(pb));
  // both tables from one walk over the rows, so a cut piece has one slot
  std::vector<int32_t> tab, all, cut;
  std::vector<uint8_t> is_heavy((size_t)p->mb, 0);
  for (int32_t r : heavy) is_heavy[r] = 1;
  int32_t slots = 0;
  for (int32_t r = 0; r < p->mb; ++r) {
    const int64_t lo = rp[r], len = rp[r + 1] - lo;
    int64_t C = len > piece ? ceil_div(len, piece) : 1;
    int64_t sz = C > 1 ? (ceil_div(len, C) + 1) & ~(int64_t)1 : std::max<int64_t>(len, 1);  // whole pairs
    C = C > 1 ? ceil_div(len, sz) : 1;
    for (int64_t c = 0; c < C; ++c) {
      const int32_t e[8] = {r, (int32_t)(lo + c * sz), (int32_t)std::min(lo + len, lo + (c + 1) * sz),
                            C > 1 ? slots + (int32_t)c : 0, (int32_t)c, (int32_t)C, 0, 0};
      all.insert(all.end(), e, e + 8);
      if (is_heavy[r]) tab.insert(tab.end(), e, e + 8);
    }
    if (C > 1) {
      const int32_t e[4] = {r, slots, (int32_t)C, 0};
      cut.insert(cut.end(), e, e + 4);
      slots += (int32_t)C;
    }
  }
  if (slots == 0) return SPMM_OK;
  if ((st = dev_alloc(&p->pieces, (int64_t)tab.size())) != SPMM_OK) return st;
  if ((st = dev_alloc(&p->pieces_all, (int64_t)all.size())) != SPMM_OK) return st;
  if ((st = dev_alloc(&p->cut_rows, (int64_t)cut.size())) != SPMM_OK) return st;
  SPMM_HIP(hipMemcpy(p->cut_rows, cut.data(), sizeof(int32_t) * cut.size(), hipMemcpyHostToDevice));
  p->num_cut = (int32_t)(cut.size() / 4);
  SPMM_HIP(hipMemcpy(p->pieces, tab.data(), sizeof(int32_t) * tab.size(), hipMemcpyHostToDevice));
  SPMM_HIP(hipMemcpy(p->pieces_all, all.data(), sizeof(int32_t) * all.size(), hipMemcpyHostToDevice));
  p->num_pieces = (int32_t)(tab.size() / 8);
  // split rows of very different lengths: the four-wave split alone leaves
  // the longest far behind the others
  std::vector<int64_t> lens;
  for (int32_t r : heavy) lens.push_back(rp[r + 1] - rp[r]);
  std::nth_element(lens.begin(), lens.begin() + lens.size() / 2, lens.end());
  p->pieces_spread = longest >= 2 * lens[lens.size() / 2];
  p->num_pieces_all = (int32_t)(all.size() / 8);
  p->num_slots = slots;
  return SPMM_OK;
}

// The piece workspace of a plan for runs of up to n columns, at any tile
// width: partials of num_slots x 16 rows x n (rounded up to 128) FP32. Grows
// under a lock, after the device has finished the launches that may still
// use the old one. False when it cannot grow now (the stream is being
// captured, or allocation failed): the run then splits its long rows over one
// workgroup each.
static std::mutex g_piece_mu;
static bool piece_workspace(const spmm_plan_s* cp, int64_t n, hipStream_t s) {
  spmm_plan_s* p = const_cast<spmm_plan_s*>(cp);
  std::lock_guard<std::mutex> lk(g_piece_mu);
  if (p->piece_ws_n >= n) return true;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return false;
  const int64_t cap = std::max<int64_t>(n, 2 * p->piece_ws_n);
  const int64_t part_bytes = (int64_t)p->num_slots * 16 * (ceil_div(cap, 128) * 128) * 4;
  if (p->piece_part) {
    if (hipDeviceSynchronize() != hipSuccess) return false;
    (void)hipFree(p->piece_part);
    p->piece_part = nullptr;
    p->piece_ws_n = 0;
    p->piece_ws_bytes = 0;
  }
  if (hipMalloc((void**)&p->piece_part, (size_t)part_bytes) != hipSuccess) {
    p->piece_part = nullptr;
    return false;
  }
  p->piece_ws_n = cap;
  p->piece_ws_bytes = part_bytes;
  return true;
}

}  // namespace spmm

using namespace spmm;

struct spmm_dyn_s {
  int64_t m = 0, k = 0;
  int32_t b = 0, mb = 0, kb = 0;
  int64_t max_nnzb = 0;
  spmm_dtype_t w = SPMM_F32, x = SPMM_F32, y = SPMM_F32;
  Geometry geo{};
  PlanBuffers pb;
  int32_t* status = nullptr;   // internal status word (device)
  int32_t* nnz_last = nullptr; // device copy of the last call's nnz
  void* packed = nullptr;      // values gathered into block-CSR order, sized for max_nnzb
  float* packed_scales = nullptr;
  int device = 0;
  bool ran = false;
  bool panels_current = false;  // panel_ptr matches the last call's row_ptr
  int32_t tuned[32] = {};       // tuned compute variant per n class, 0 = none
};

extern "C" {

const char* spmm_last_error(void) { return g_last_error.c_str(); }

spmm_status_t spmm_plan_static(int64_t m, int64_t k, int32_t b, const uint8_t* block_mask_host, spmm_dtype_t w,
                               spmm_dtype_t x, spmm_dtype_t y, const spmm_plan_opts* opts, spmm_plan_t* out) {
  clear_error();
  if (!out) return fail(SPMM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (m < 1 || k < 1) return fail(SPMM_ERR_INVALID_ARG, "m and k must be positive");
  if (!valid_static_block(b)) return fail(SPMM_ERR_INVALID_ARG, "block size must be one of 1, 4, 8, 16, 32, 64");
  if (!block_mask_host) return fail(SPMM_ERR_INVALID_ARG, "block mask is NULL");
  if (!dtype_triple_supported(w, x, y)) return fail(SPMM_ERR_UNSUPPORTED, "unsupported dtype combination");
  if (b == 64 && x != SPMM_F16 && x != SPMM_BF16) return fail(SPMM_ERR_UNSUPPORTED, "b = 64 needs FP16 or BF16 X");
  if (m > INT32_MAX / 2 || k > INT32_MAX / 2) return fail(SPMM_ERR_UNSUPPORTED, "m or k too large");
  const int64_t mb = ceil_div(m, b), kb = ceil_div(k, b);
  int64_t nnzb = 0;
  for (int64_t i = 0; i < mb * kb; ++i) nnzb += block_mask_host[i] != 0;
  if (nnzb > INT32_MAX / 2) return fail(SPMM_ERR_UNSUPPORTED, "too many nonzero blocks");
  if (opts && (opts->group_rows < 0 || opts->num_panels < 0))
    return fail(SPMM_ERR_INVALID_ARG, "negative plan option");
  if (opts && variant_form(opts->variant) == 5)
    return fail(SPMM_ERR_INVALID_ARG, "variant form 5 (one launch) is for dynamic calls");
  if (opts && !valid_variant(b, opts->variant))
    return fail(SPMM_ERR_INVALID_ARG, "variant must be 0 or (2, 4, 8 or 0) + 256 x (0 .. 4); 2 needs b >= 16");
  if (opts && (opts->dense_dispatch < 0 || opts->dense_dispatch > 2))
    return fail(SPMM_ERR_INVALID_ARG, "dense_dispatch must be 0, 1 or 2");
  const int32_t dense_opt = opts ? opts->dense_dispatch : 0;
  if (dense_opt && !dense_dispatch_eligible(w, x, y))
    return fail(SPMM_ERR_UNSUPPORTED, "dense dispatch needs W in the 16-bit X type and Y in it or FP32");
  double predicted = 0.0;
  {
    const double d = mb * kb > 0 ? (double)nnzb / ((double)mb * (double)kb) : 0.0;
    const int64_t feat = std::max<int64_t>(1, std::llround(std::sqrt((double)m * (double)k)));
    if (d > 0.0 && spmm_speedup_model(feat, d, b, &predicted) != SPMM_OK) predicted = 0.0;
    clear_error();
  }
  const bool keep_dense = dense_opt == 2 || (dense_opt == 1 && nnzb > 0 && predicted < 1.0);
  if (opts && variant_form(opts->variant) == 3 && !keep_dense)
    return fail(SPMM_ERR_INVALID_ARG, "variant form 3 (dense) needs a plan that keeps a dense copy");

  spmm_plan_s* p = new (std::nothrow) spmm_plan_s;
  if (!p) return fail(SPMM_ERR_OOM, "host allocation failed");
  p->m = m; p->k = k; p->b = b; p->mb = (int32_t)mb; p->kb = (int32_t)kb; p->nnzb = nnzb;
  p->w = w; p->x = x; p->y = y;
  p->variant_opt = opts ? opts->variant : 0;
  p->predicted_speedup = predicted;
  p->dense_mode = keep_dense ? dense_opt : 0;
  p->geo = choose_geometry(m, k, b, nnzb, opts ? opts->n_hint : 0, opts, device_cu_count(), x);
  spmm_status_t st = SPMM_OK;
  uint8_t* mask_dev = nullptr;
  hipStream_t s = nullptr;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) st = fail_hip(e, "hipGetDevice");
  if (st == SPMM_OK) st = alloc_plan_buffers(p->pb, p->geo, (int32_t)mb, nnzb, false);
  if (st == SPMM_OK) st = dev_alloc(&mask_dev, mb * kb);
  if (st == SPMM_OK) {  // plan-owned values in block-CSR order
    const int64_t vbytes = nnzb * (int64_t)b * b * dtype_bytes(w);
    e = hipMalloc(&p->values, (size_t)std::max<int64_t>(vbytes, 16));
    if (e != hipSuccess) st = fail_hip(e, "hipMalloc values");
  }
  if (st == SPMM_OK && w == SPMM_FP8_E4M3) st = dev_alloc(&p->scales, nnzb);
  if (st == SPMM_OK && (e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess)
    st = fail_hip(e, "hipStreamCreate");
  if (st == SPMM_OK && (e = hipMemcpyAsync(mask_dev, block_mask_host, (size_t)(mb * kb), hipMemcpyHostToDevice, s)) != hipSuccess)
    st = fail_hip(e, "mask upload");
  if (st == SPMM_OK) st = build_static_plan(mask_dev, (int32_t)mb, (int32_t)kb, p->geo, p->pb, s);
  if (st == SPMM_OK && (e = hipStreamSynchronize(s)) != hipSuccess) st = fail_hip(e, "plan build");
  const bool sddmm = b <= 32 && (x == SPMM_F16 || x == SPMM_BF16);
  if (st == SPMM_OK && (b >= 16 || sddmm)) {
    // host copy of the row pointers: long rows to split, SDDMM tasks
    std::vector<int32_t> rp((size_t)mb + 1);
    e = hipMemcpy(rp.data(), p->pb.row_ptr, sizeof(int32_t) * rp.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) st = fail_hip(e, "row pointer download");
    if (st == SPMM_OK && b == 16 && x != SPMM_F32) st = classify_heavy_rows(p, rp);
    if (st == SPMM_OK && sddmm) st = build_sddmm_tasks(p, rp);
    if (st == SPMM_OK && sddmm) st = build_sddmm_tiled(p, rp);
  }
  if (s) (void)hipStreamDestroy(s);
  if (mask_dev) (void)hipFree(mask_dev);
  if (st != SPMM_OK) {
    free_plan_buffers(p->pb);
    if (p->values) (void)hipFree(p->values);
    if (p->scales) (void)hipFree(p->scales);
    if (p->light_rows) (void)hipFree(p->light_rows);
    if (p->heavy_rows) (void)hipFree(p->heavy_rows);
    if (p->pieces) (void)hipFree(p->pieces);
    if (p->pieces_all) (void)hipFree(p->pieces_all);
    if (p->cut_rows) (void)hipFree(p->cut_rows);
    if (p->sddmm_tasks) (void)hipFree(p->sddmm_tasks);
    if (p->sddmm_tiled_tasks) (void)hipFree(p->sddmm_tiled_tasks);
    if (p->sddmm_tiled_ent) (void)hipFree(p->sddmm_tiled_ent);
    if (p->ell_slot) (void)hipFree(p->ell_slot);
    delete p;
    return st;
  }
  *out = p;
  return SPMM_OK;
}

spmm_status_t spmm_plan_set_values(spmm_plan_t p, const void* values_dev, const float* scales_dev, void* stream) {
  clear_error();
  if (!p) return fail(SPMM_ERR_INVALID_ARG, "plan is NULL");
  if (p->nnzb > 0 && !values_dev) return fail(SPMM_ERR_INVALID_ARG, "values are NULL");
  if (p->w == SPMM_FP8_E4M3 && p->nnzb > 0 && !scales_dev) return fail(SPMM_ERR_INVALID_ARG, "FP8 weights need block scales");
  if (p->w != SPMM_FP8_E4M3 && scales_dev) return fail(SPMM_ERR_INVALID_ARG, "block scales are only for FP8 weights");
  spmm_status_t st = check_device(p->device);
  if (st != SPMM_OK) return st;
  st = copy_values_csr(p->pb.col_idx, p->nnzb, p->b, (int32_t)p->k, values_dev, p->values, dtype_bytes(p->w),
                       scales_dev, p->scales, (hipStream_t)stream);
  if (st != SPMM_OK) return st;
  if (p->dense_mode && (st = build_dense_copy(p, (hipStream_t)stream)) != SPMM_OK) return st;
  p->has_values = true;
  return SPMM_OK;
}

// Candidate variants of the plan's kernels (tile widths times forms).
static int plan_candidates(const spmm_plan_s* p, int32_t (&c)[8]) {
  int k = 0;
  if (plan_uses_row_kernel(p)) {
    for (int32_t ns : {2, 4, 8}) c[k++] = make_variant(ns, 1);
    if (p->w == p->x && p->num_heavy == 0 && p->b <= 32)
      for (int32_t ns : {2, 4, 8}) c[k++] = make_variant(ns, 2);
    if (p->b == 16) c[k++] = make_variant(0, 4);
  } else if (p->b < 16 && p->x != SPMM_F32) {
    c[k++] = make_variant(4, 1);
    c[k++] = make_variant(8, 1);
    if (small_lds_eligible(p->b, p->w, p->x)) c[k++] = make_variant(0, 2);
  }
  if (p->dense_w) c[k++] = make_variant(0, 3);
  return k;
}

// Times every candidate on the caller's operands (after 8 + nc untimed runs,
// 5 interleaved rounds of one launch per candidate, HIP events on `s`, the
// median per candidate), records the fastest for n's class in the plan and
// the process table, and leaves Y holding its result. Synchronises `s`.
static spmm_status_t tune_plan(spmm_plan_s* p, int64_t n, const void* X, int64_t ldx, void* Y, int64_t ldy,
                               hipStream_t s, int32_t* cand_out, float* times_out, int32_t* count_out,
                               int32_t* best_out) {
  int32_t cand[8];
  const int nc = plan_candidates(p, cand);
  float times[8];
  int32_t best = 0;
  float best_ms = 0.f;
  spmm_status_t st = SPMM_OK;
  if (nc > 0) {
    // The clocks ramp up over the first launches of a process: warm up with
    // the first candidate, run every candidate once untimed, then time the
    // candidates in interleaved rounds (one launch each per round, its own
    // pair of events) and keep each one's median, so that no candidate is
    // favoured by running later.
    constexpr int kRounds = 5;
    for (int i = 0; i < 8 && st == SPMM_OK; ++i) st = run_plan(p, n, X, ldx, Y, ldy, cand[0], false, s);
    for (int c = 0; c < nc && st == SPMM_OK; ++c) st = run_plan(p, n, X, ldx, Y, ldy, cand[c], false, s);
    if (st != SPMM_OK) return st;
    hipEvent_t ev[16] = {};
    hipError_t he = hipSuccess;
    for (int i = 0; i < 2 * nc && he == hipSuccess; ++i) he = hipEventCreate(&ev[i]);
    float samples[8][kRounds] = {};
    for (int r = 0; r < kRounds && st == SPMM_OK && he == hipSuccess; ++r) {
      for (int c = 0; c < nc && st == SPMM_OK && he == hipSuccess; ++c) {
        he = hipEventRecord(ev[2 * c], s);
        if (he == hipSuccess) st = run_plan(p, n, X, ldx, Y, ldy, cand[c], false, s);
        if (he == hipSuccess && st == SPMM_OK) he = hipEventRecord(ev[2 * c + 1], s);
      }
      if (he == hipSuccess && st == SPMM_OK) he = hipEventSynchronize(ev[2 * nc - 1]);
      for (int c = 0; c < nc && he == hipSuccess && st == SPMM_OK; ++c)
        he = hipEventElapsedTime(&samples[c][r], ev[2 * c], ev[2 * c + 1]);
    }
    for (int i = 0; i < 2 * nc; ++i)
      if (ev[i]) (void)hipEventDestroy(ev[i]);
    if (st != SPMM_OK) return st;
    if (he != hipSuccess) return fail_hip(he, "autotune timing");
    for (int c = 0; c < nc; ++c) {
      std::sort(samples[c], samples[c] + kRounds);
      times[c] = samples[c][kRounds / 2];
      if (!best || times[c] < best_ms) {
        best = cand[c];
        best_ms = times[c];
      }
    }
    // leave Y holding the result of the chosen variant
    if ((st = run_plan(p, n, X, ldx, Y, ldy, best, false, s)) != SPMM_OK) return st;
    SPMM_HIP(hipStreamSynchronize(s));
    p->tuned[n_class(n)] = best;
    tune_table_put(p, n, best);
  } else {
    if ((st = run_plan(p, n, X, ldx, Y, ldy, 0, false, s)) != SPMM_OK) return st;
    SPMM_HIP(hipStreamSynchronize(s));
  }
  for (int c = 0; c < nc; ++c) {
    if (cand_out) cand_out[c] = cand[c];
    if (times_out) times_out[c] = times[c];
  }
  if (count_out) *count_out = nc;
  if (best_out) *best_out = best;
  return SPMM_OK;
}

static spmm_status_t check_run_args(const spmm_plan_s* p, int64_t n, const void* X, int64_t ldx, const void* Y,
                                    int64_t ldy) {
  if (n > INT32_MAX / 2) return fail(SPMM_ERR_UNSUPPORTED, "n too large");
  if (!p->has_values) return fail(SPMM_ERR_INVALID_ARG, "values were not set on this plan");
  spmm_status_t st;
  if ((st = check_dense(X, ldx, n, dtype_bytes(p->x), "X")) != SPMM_OK) return st;
  if ((st = check_dense(Y, ldy, n, dtype_bytes(p->y), "Y")) != SPMM_OK) return st;
  return check_device(p->device);
}

spmm_status_t spmm_run_static(spmm_plan_t p, int64_t n, const void* X, int64_t ldx, void* Y, int64_t ldy,
                              void* stream) {
  clear_error();
  if (!p) return fail(SPMM_ERR_INVALID_ARG, "plan is NULL");
  if (n < 0) return fail(SPMM_ERR_INVALID_ARG, "n is negative");
  if (n == 0) return SPMM_OK;
  spmm_status_t st = check_run_args(p, n, X, ldx, Y, ldy);
  if (st != SPMM_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const int32_t v = plan_variant(p, n);
  if (v == 0) {
    int32_t cand[8];
    if (plan_candidates(p, cand) > 1 && tune_on_first_run(s))
      return tune_plan(p, n, X, ldx, Y, ldy, s, nullptr, nullptr, nullptr, nullptr);
  }
  return run_plan(p, n, X, ldx, Y, ldy, v, false, s);
}

spmm_status_t spmm_autotune_static(spmm_plan_t p, int64_t n, const void* X, int64_t ldx, void* Y, int64_t ldy,
                                   void* stream, int32_t* variant_out, float* times_ms_out) {
  clear_error();
  if (!p) return fail(SPMM_ERR_INVALID_ARG, "plan is NULL");
  if (n <= 0) return fail(SPMM_ERR_INVALID_ARG, "n must be positive for tuning");
  spmm_status_t st = check_run_args(p, n, X, ldx, Y, ldy);
  if (st != SPMM_OK) return st;
  int32_t cand[8], count = 0, best = 0;
  float times[8];
  if ((st = tune_plan(p, n, X, ldx, Y, ldy, (hipStream_t)stream, cand, times, &count, &best)) != SPMM_OK) return st;
  if (variant_out) *variant_out = best;
  if (times_ms_out) {  // per tile width, the best over the kernel forms
    for (int i = 0; i < 3; ++i) times_ms_out[i] = -1.f;
    for (int c = 0; c < count; ++c) {
      const int32_t ns = variant_ns(cand[c]);
      const int slot = ns == 2 ? 0 : (ns == 4 ? 1 : (ns == 8 ? 2 : -1));
      if (slot >= 0 && (times_ms_out[slot] < 0.f || times[c] < times_ms_out[slot])) times_ms_out[slot] = times[c];
    }
  }
  return SPMM_OK;
}

spmm_status_t spmm_autotune_static_all(spmm_plan_t p, int64_t n, const void* X, int64_t ldx, void* Y, int64_t ldy,
                                       void* stream, int32_t capacity, int32_t* variants, float* times_ms,
                                       int32_t* count, int32_t* best) {
  clear_error();
  if (!p) return fail(SPMM_ERR_INVALID_ARG, "plan is NULL");
  if (n <= 0) return fail(SPMM_ERR_INVALID_ARG, "n must be positive for tuning");
  if (capacity < 8 || !variants || !times_ms || !count) return fail(SPMM_ERR_INVALID_ARG, "need 8 output slots");
  spmm_status_t st = check_run_args(p, n, X, ldx, Y, ldy);
  if (st != SPMM_OK) return st;
  return tune_plan(p, n, X, ldx, Y, ldy, (hipStream_t)stream, variants, times_ms, count, best);
}

spmm_status_t spmm_autotune_clear(void) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  g_tune_loaded = true;  // not reloaded from the cache file
  return SPMM_OK;
}

spmm_status_t spmm_plan_variant(spmm_plan_t p, int64_t n, int32_t* variant) {
  clear_error();
  if (!p || !variant) return fail(SPMM_ERR_INVALID_ARG, "NULL argument");
  if (n < 0) return fail(SPMM_ERR_INVALID_ARG, "n is negative");
  *variant = plan_variant(p, n);
  return SPMM_OK;
}

spmm_status_t spmm_plan_info(spmm_plan_t p, int64_t* nnzb, int32_t* group_rows, int32_t* num_groups,
                             int32_t* num_panels, int32_t* num_split_rows) {
  clear_error();
  if (!p) return fail(SPMM_ERR_INVALID_ARG, "plan is NULL");
  if (num_split_rows) *num_split_rows = p->num_heavy;
  if (nnzb) *nnzb = p->nnzb;
  if (group_rows) *group_rows = p->geo.group_rows;
  if (num_groups) *num_groups = p->geo.num_groups;
  if (num_panels) *num_panels = p->geo.num_panels;
  return SPMM_OK;
}

spmm_status_t spmm_plan_export(spmm_plan_t p, int32_t* row_ptr, int32_t* col_idx, int32_t* panel_ptr,
                               int32_t* order) {
  clear_error();
  if (!p) return fail(SPMM_ERR_INVALID_ARG, "plan is NULL");
  spmm_status_t st = check_device(p->device);
  if (st != SPMM_OK) return st;
  SPMM_HIP(hipDeviceSynchronize());
  if (row_ptr) SPMM_HIP(hipMemcpy(row_ptr, p->pb.row_ptr, sizeof(int32_t) * (p->mb + 1), hipMemcpyDeviceToHost));
  if (col_idx && p->nnzb)
    SPMM_HIP(hipMemcpy(col_idx, p->pb.col_idx, sizeof(int32_t) * p->nnzb, hipMemcpyDeviceToHost));
  if (panel_ptr)
    SPMM_HIP(hipMemcpy(panel_ptr, p->pb.panel_ptr, sizeof(int32_t) * (p->geo.num_panels + 1), hipMemcpyDeviceToHost));
  if (order && p->nnzb) SPMM_HIP(hipMemcpy(order, p->pb.order, sizeof(int32_t) * p->nnzb, hipMemcpyDeviceToHost));
  return SPMM_OK;
}

spmm_status_t spmm_plan_destroy(spmm_plan_t p) {
  clear_error();
  if (!p) return SPMM_OK;
  free_plan_buffers(p->pb);
  if (p->values) (void)hipFree(p->values);
  if (p->scales) (void)hipFree(p->scales);
  if (p->light_rows) (void)hipFree(p->light_rows);
  if (p->heavy_rows) (void)hipFree(p->heavy_rows);
  if (p->pieces) (void)hipFree(p->pieces);
  if (p->pieces_all) (void)hipFree(p->pieces_all);
  if (p->cut_rows) (void)hipFree(p->cut_rows);
  if (p->piece_part) (void)hipFree(p->piece_part);
  if (p->sddmm_dense_ws) (void)hipFree(p->sddmm_dense_ws);
  if (p->sddmm_tasks) (void)hipFree(p->sddmm_tasks);
  if (p->ell_slot) (void)hipFree(p->ell_slot);
  if (p->dense_w) (void)hipFree(p->dense_w);
  if (p->sddmm_tiled_tasks) (void)hipFree(p->sddmm_tiled_tasks);
  if (p->sddmm_tiled_ent) (void)hipFree(p->sddmm_tiled_ent);
  delete p;
  return SPMM_OK;
}

spmm_status_t spmm_plan_memory(spmm_plan_t p, int64_t* device_bytes, int64_t* value_bytes) {
  clear_error();
  if (!p) return fail(SPMM_ERR_INVALID_ARG, "plan is NULL");
  auto n1 = [](int64_t c) { return std::max<int64_t>(c, 1); };  // as dev_alloc rounds
  const int64_t nnz = p->nnzb;
  int64_t idx = 4 * n1((int64_t)p->geo.num_panels + 1) + 4 * n1((int64_t)p->mb + 1) + 4 * n1(nnz) +
                4 * (p->pb.order ? n1(nnz) : 0) + 4 * n1(p->pb.scratch_ints) + 8 * n1((int64_t)p->geo.num_groups + 1);
  if (p->light_rows) idx += 4 * n1((int64_t)p->mb - p->num_heavy);
  if (p->heavy_rows) idx += 4 * n1(p->num_heavy);
  if (p->pieces) idx += 32 * (n1(p->num_pieces) + n1(p->num_pieces_all)) + 16 * n1(p->num_cut);
  idx += p->piece_ws_bytes + p->sddmm_dense_ws_bytes;
  if (p->sddmm_tasks) idx += 8 * n1(p->sddmm_num_tasks);
  if (p->sddmm_tiled_tasks) idx += 16 * n1(p->sddmm_tiled_num) + 8 * n1(nnz);
  if (p->ell_slot) idx += 4 * n1(nnz);
  const int64_t vals = std::max<int64_t>(nnz * (int64_t)p->b * p->b * dtype_bytes(p->w), 16) +
                       (p->scales ? 4 * n1(nnz) : 0);
  const int64_t dense = p->dense_w ? p->m * p->k * (int64_t)dtype_bytes(p->w) : 0;
  if (device_bytes) *device_bytes = idx + vals + dense;
  if (value_bytes) *value_bytes = vals;
  return SPMM_OK;
}

spmm_status_t spmm_plan_dispatch(spmm_plan_t p, double* predicted_speedup, int32_t* has_dense) {
  clear_error();
  if (!p) return fail(SPMM_ERR_INVALID_ARG, "plan is NULL");
  if (predicted_speedup) *predicted_speedup = p->predicted_speedup;
  if (has_dense) *has_dense = p->dense_mode ? 1 : 0;
  return SPMM_OK;
}

// ------------------------------------------------------------------ dynamic
spmm_status_t spmm_dynamic_create(int64_t m, int64_t k, int32_t b, int64_t max_nnzb, spmm_dtype_t w, spmm_dtype_t x,
                                  spmm_dtype_t y, const spmm_plan_opts* opts, spmm_dyn_t* out) {
  clear_error();
  if (!out) return fail(SPMM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (m < 1 || k < 1) return fail(SPMM_ERR_INVALID_ARG, "m and k must be positive");
  if (!valid_block(b)) return fail(SPMM_ERR_INVALID_ARG, "block size must be one of 1, 4, 8, 16, 32");
  if (max_nnzb < 0) return fail(SPMM_ERR_INVALID_ARG, "max_nnzb is negative");
  if (!dtype_triple_supported(w, x, y)) return fail(SPMM_ERR_UNSUPPORTED, "unsupported dtype combination");
  if (m > INT32_MAX / 2 || k > INT32_MAX / 2 || max_nnzb > INT32_MAX / 4)
    return fail(SPMM_ERR_UNSUPPORTED, "size too large");
  if (opts && (opts->group_rows < 0 || opts->num_panels < 0)) return fail(SPMM_ERR_INVALID_ARG, "negative plan option");
  spmm_dyn_s* h = new (std::nothrow) spmm_dyn_s;
  if (!h) return fail(SPMM_ERR_OOM, "host allocation failed");
  h->m = m; h->k = k; h->b = b;
  h->mb = (int32_t)ceil_div(m, b);
  h->kb = (int32_t)ceil_div(k, b);
  h->max_nnzb = max_nnzb;
  h->w = w; h->x = x; h->y = y;
  h->geo = choose_geometry(m, k, b, max_nnzb, opts ? opts->n_hint : 0, opts, device_cu_count(), x);
  spmm_status_t st = SPMM_OK;
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) st = fail_hip(e, "hipGetDevice");
  if (st == SPMM_OK) st = alloc_plan_buffers(h->pb, h->geo, h->mb, max_nnzb, true);
  if (st == SPMM_OK) st = dev_alloc(&h->status, 2);
  if (st == SPMM_OK) st = dev_alloc(&h->nnz_last, 2);
  if (st == SPMM_OK) {
    const int64_t vbytes = max_nnzb * (int64_t)b * b * dtype_bytes(w);
    e = hipMalloc(&h->packed, (size_t)std::max<int64_t>(vbytes, 16));
    if (e != hipSuccess) st = fail_hip(e, "hipMalloc packed values");
  }
  if (st == SPMM_OK && w == SPMM_FP8_E4M3) st = dev_alloc(&h->packed_scales, max_nnzb);
  if (st == SPMM_OK) {
    if ((e = hipMemset(h->status, 0, 2 * sizeof(int32_t))) != hipSuccess) st = fail_hip(e, "hipMemset");
  }
  if (st != SPMM_OK) {
    free_plan_buffers(h->pb);
    if (h->status) (void)hipFree(h->status);
    if (h->nnz_last) (void)hipFree(h->nnz_last);
    if (h->packed) (void)hipFree(h->packed);
    if (h->packed_scales) (void)hipFree(h->packed_scales);
    delete h;
    return st;
  }
  *out = h;
  return SPMM_OK;
}

spmm_status_t spmm_run_dynamic(spmm_dyn_t h, const int32_t* nnzb_dev, const int32_t* rows, const int32_t* cols,
                               const void* values_dev, const float* scales_dev, int64_t n, const void* X, int64_t ldx,
                               void* Y, int64_t ldy, int32_t* status_dev, void* stream) {
  clear_error();
  if (!h) return fail(SPMM_ERR_INVALID_ARG, "handle is NULL");
  if (!nnzb_dev || !status_dev) return fail(SPMM_ERR_INVALID_ARG, "nnzb_dev and status_dev are required");
  if (h->max_nnzb > 0 && (!rows || !cols || !values_dev))
    return fail(SPMM_ERR_INVALID_ARG, "index and value buffers are required");
  if (h->w == SPMM_FP8_E4M3 && h->max_nnzb > 0 && !scales_dev) return fail(SPMM_ERR_INVALID_ARG, "FP8 weights need block scales");
  if (h->w != SPMM_FP8_E4M3 && scales_dev) return fail(SPMM_ERR_INVALID_ARG, "block scales are only for FP8 weights");
  if (n < 0) return fail(SPMM_ERR_INVALID_ARG, "n is negative");
  if (n > INT32_MAX / 2) return fail(SPMM_ERR_UNSUPPORTED, "n too large");
  spmm_status_t st;
  if (n > 0) {
    if ((st = check_dense(X, ldx, n, dtype_bytes(h->x), "X")) != SPMM_OK) return st;
    if ((st = check_dense(Y, ldy, n, dtype_bytes(h->y), "Y")) != SPMM_OK) return st;
  }
  if (((uintptr_t)values_dev) % 16 != 0) return fail(SPMM_ERR_INVALID_ARG, "values are not 16-byte aligned");
  if ((st = check_device(h->device)) != SPMM_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  // re-bucket into block-CSR and run the block-CSR kernel (the same kernel and
  // order as a static plan of the same pattern). Small capacities encode in
  // one workgroup and leave the values in place (read through csr_src); edge
  // blocks that cross k need the copying path, which zeroes their tail. Or, in
  // one launch, encode and multiply together (variant form 5).
  const int want = requested_builder();
  const bool in_place = h->k % h->b == 0 && want != kBuilderMulti;
  const bool rows_fit = dynamic_rows_fits((int32_t)h->max_nnzb, h->mb, h->kb);
  const bool one_fit = dynamic_small_fits((int32_t)h->max_nnzb, h->mb, h->kb, h->geo.num_groups);
  int builder = kBuilderMulti;
  if (in_place && rows_fit && want != kBuilderOne) builder = kBuilderRows;
  else if (in_place && one_fit) builder = kBuilderOne;
  else if (in_place && rows_fit) builder = kBuilderRows;
  const bool one_wg = builder != kBuilderMulti;  // values read in place through csr_src
  const bool fused_ok = n > 0 && want == kBuilderNone &&
                        dynamic_fused_eligible(h->b, h->w, h->x, h->y, h->k, h->mb, h->kb, h->max_nnzb);
  auto encode = [&]() -> spmm_status_t {
    if (builder == kBuilderRows)
      return build_dynamic_csr_rows(nnzb_dev, rows, cols, (int32_t)h->max_nnzb, h->mb, h->kb, h->pb, h->status,
                                    status_dev, h->nnz_last, s);
    if (builder == kBuilderOne)
      return build_dynamic_csr_small(nnzb_dev, rows, cols, (int32_t)h->max_nnzb, h->mb, h->kb, h->geo, h->pb,
                                     h->status, status_dev, h->nnz_last, s);
    return build_dynamic_csr(nnzb_dev, rows, cols, (int32_t)h->max_nnzb, h->mb, h->kb, h->b, (int32_t)h->k, h->geo,
                             h->pb, values_dev, h->packed, dtype_bytes(h->w), scales_dev, h->packed_scales, h->status,
                             status_dev, h->nnz_last, s);
  };
  if (n == 0) {  // the encode alone (status, export)
    if ((st = encode()) != SPMM_OK) return st;
    h->ran = true;
    h->panels_current = builder != kBuilderRows;
    return SPMM_OK;
  }
  RunArgs a{};
  a.plan = kernel_plan(h->m, h->k, h->b, h->mb, h->kb, h->geo, h->pb);
  a.W = one_wg ? values_dev : h->packed;
  a.scales = one_wg ? scales_dev : h->packed_scales;
  a.w_index = one_wg ? h->pb.csr_src : nullptr;
  a.X = X;
  a.Y = Y;
  a.ldx = ldx;
  a.ldy = ldy;
  a.n = (int32_t)n;
  a.wt = h->w;
  a.xt = h->x;
  a.yt = h->y;
  a.status = h->status;
  a.nnz = h->max_nnzb;
  // one call with a variant: the one-launch form, else the encoder and then
  // the compute kernel's form
  auto call = [&](int32_t v) -> spmm_status_t {
    if (variant_form(v) == 5 && fused_ok) {
      RunArgs f = a;
      f.W = values_dev;
      f.ns = variant_ns(v) ? variant_ns(v) : default_ns(n);
      h->panels_current = false;
      return launch_dynamic_fused(f, nnzb_dev, rows, cols, (int32_t)h->max_nnzb, h->kb, h->pb.row_ptr,
                                  h->pb.col_idx, h->pb.csr_src, h->status, status_dev, h->nnz_last, s);
    }
    spmm_status_t e = encode();
    if (e != SPMM_OK) return e;
    h->panels_current = builder != kBuilderRows;
    RunArgs t = a;
    return run_dynamic_kernel(t, h->pb.row_ptr, h->pb.col_idx, s, variant_form(v) == 5 ? 0 : v);
  };
  h->ran = true;
  // the first call of an n class times every candidate on this call's
  // operands, encoder included (the call is idempotent; the status word makes
  // every candidate skip a failed encode alike), as a static plan's first run
  // times its variants
  const int nc = n_class(n);
  if (!h->tuned[nc] && tune_on_first_run(s)) {
    int32_t cand[10];
    const int ncand = dynamic_candidates(h->b, h->w, h->x, fused_ok, cand);
    if (ncand > 1) {
      // as tune_plan: warm-up calls, then interleaved rounds (three calls per
      // candidate per round, their own pair of events), the median per candidate
      constexpr int kRounds = 5, kCalls = 3;
      for (int i = 0; i < 8 && st == SPMM_OK; ++i) st = call(cand[0]);
      for (int c = 0; c < ncand && st == SPMM_OK; ++c) st = call(cand[c]);
      if (st != SPMM_OK) return st;
      hipEvent_t ev[20] = {};
      hipError_t he = hipSuccess;
      for (int i = 0; i < 2 * ncand && he == hipSuccess; ++i) he = hipEventCreate(&ev[i]);
      float samples[10][kRounds] = {};
      for (int r = 0; r < kRounds && st == SPMM_OK && he == hipSuccess; ++r) {
        for (int c = 0; c < ncand && st == SPMM_OK && he == hipSuccess; ++c) {
          he = hipEventRecord(ev[2 * c], s);
          for (int i = 0; i < kCalls && st == SPMM_OK && he == hipSuccess; ++i) st = call(cand[c]);
          if (he == hipSuccess && st == SPMM_OK) he = hipEventRecord(ev[2 * c + 1], s);
        }
        if (he == hipSuccess && st == SPMM_OK) he = hipEventSynchronize(ev[2 * ncand - 1]);
        for (int c = 0; c < ncand && he == hipSuccess && st == SPMM_OK; ++c)
          he = hipEventElapsedTime(&samples[c][r], ev[2 * c], ev[2 * c + 1]);
      }
      for (int i = 0; i < 2 * ncand; ++i)
        if (ev[i]) (void)hipEventDestroy(ev[i]);
      if (st != SPMM_OK) return st;
      if (he != hipSuccess) return fail_hip(he, "dynamic tuning");
      int32_t best = 0;
      float best_ms = 0.f;
      for (int c = 0; c < ncand; ++c) {
        std::sort(samples[c], samples[c] + kRounds);
        const float ms = samples[c][kRounds / 2];
        if (!best || ms < best_ms) {
          best = cand[c];
          best_ms = ms;
        }
      }
      int32_t enc = 0;  // a failed encode skipped every candidate: nothing was measured
      SPMM_HIP(hipMemcpy(&enc, h->status, sizeof(int32_t), hipMemcpyDeviceToHost));
      if (enc == 0) h->tuned[nc] = best;
    }
  }
  int32_t v = h->tuned[nc];
  if (const char* dv = getenv("SPMM_DYN_VARIANT")) {  // a fixed variant (comparisons, tests)
    const int32_t fv = (int32_t)atoi(dv);
    if (valid_variant(h->b, fv)) v = fv;
  }
  if (!v && fused_ok) {  // the rule: one launch where the every-row split form is the rule and the grid is small
    if (split_all_preferred(h->b, h->mb, n, default_ns(n), h->max_nnzb, device_cu_count()) &&
        dynamic_fused_preferred(h->mb, n, h->max_nnzb))
      v = make_variant(dynamic_fused_ns(n), 5);
  }
  return call(v);
}

spmm_status_t spmm_dynamic_export(spmm_dyn_t h, int32_t* row_ptr, int32_t* col_idx, int32_t* src, int32_t* panel_ptr,
                                  int64_t* nnzb) {
  clear_error();
  if (!h) return fail(SPMM_ERR_INVALID_ARG, "handle is NULL");
  if (!h->ran) return fail(SPMM_ERR_INVALID_ARG, "no dynamic call has run on this handle");
  spmm_status_t st = check_device(h->device);
  if (st != SPMM_OK) return st;
  if (!h->panels_current && panel_ptr) {  // the row-range encoder leaves the panels to the export
    SPMM_HIP(hipDeviceSynchronize());
    if ((st = dyn_panels(h->geo, h->mb, h->pb, h->status, nullptr)) != SPMM_OK) return st;
    h->panels_current = true;
  }
  SPMM_HIP(hipDeviceSynchronize());
  int32_t status = 0, nnz = 0;
  SPMM_HIP(hipMemcpy(&status, h->status, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (status != 0) return fail((spmm_status_t)status, "the last dynamic call failed on the device");
  SPMM_HIP(hipMemcpy(&nnz, h->nnz_last, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (nnzb) *nnzb = nnz;
  if (row_ptr) SPMM_HIP(hipMemcpy(row_ptr, h->pb.row_ptr, sizeof(int32_t) * (h->mb + 1), hipMemcpyDeviceToHost));
  if (col_idx && nnz) SPMM_HIP(hipMemcpy(col_idx, h->pb.col_idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
  if (src && nnz) SPMM_HIP(hipMemcpy(src, h->pb.csr_src, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
  if (panel_ptr)
    SPMM_HIP(hipMemcpy(panel_ptr, h->pb.panel_ptr, sizeof(int32_t) * (h->geo.num_panels + 1), hipMemcpyDeviceToHost));
  return SPMM_OK;
}

spmm_status_t spmm_dynamic_info(spmm_dyn_t h, int32_t* group_rows, int32_t* num_groups, int32_t* num_panels) {
  clear_error();
  if (!h) return fail(SPMM_ERR_INVALID_ARG, "handle is NULL");
  if (group_rows) *group_rows = h->geo.group_rows;
  if (num_groups) *num_groups = h->geo.num_groups;
  if (num_panels) *num_panels = h->geo.num_panels;
  return SPMM_OK;
}

spmm_status_t spmm_dynamic_destroy(spmm_dyn_t h) {
  clear_error();
  if (!h) return SPMM_OK;
  free_plan_buffers(h->pb);
  if (h->status) (void)hipFree(h->status);
  if (h->nnz_last) (void)hipFree(h->nnz_last);
  if (h->packed) (void)hipFree(h->packed);
  if (h->packed_scales) (void)hipFree(h->packed_scales);
  delete h;
  return SPMM_OK;
}

}  // extern "C"
