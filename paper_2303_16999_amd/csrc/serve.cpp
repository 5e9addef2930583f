// Serving loop (C ABI): continuous batching of requests through a chain of
// resident sparse layers, or the plain one-request-at-a-time reference path.
//
// The scheduler is host C++: a FIFO of submitted requests, an activation pool
// with first-fit allocation, the set of admitted requests and a completion
// list. A step admits from the FIFO head while memory and max_active allow,
// then advances every admitted request by one layer in one grouped launch
// (CONTINUOUS) or runs one whole request layer by layer (PLAIN).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using namespace spmm;

namespace {

double now_s() {
  using clk = std::chrono::steady_clock;
  return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

// ReLU in place over rows x n of a row-major matrix (the plain path's separate pass).
template <typename T>
__global__ void k_relu(T* __restrict__ a, int64_t rows, int64_t n, int64_t ld) {
  const int64_t total = rows * n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / n, c = i - r * n;
    T* p = a + r * ld + c;
    const float v = (float)*p;
    if (!(v > 0.f)) *p = T(0.f);
  }
}

spmm_status_t launch_relu(spmm_dtype_t t, void* a, int64_t rows, int64_t n, int64_t ld, hipStream_t s) {
  const int64_t total = rows * n;
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, ceil_div(total, 256)));
  if (t == SPMM_F16) hipLaunchKernelGGL(k_relu<_Float16>, dim3(grid), dim3(256), 0, s, (_Float16*)a, rows, n, ld);
  else if (t == SPMM_BF16) hipLaunchKernelGGL(k_relu<__bf16>, dim3(grid), dim3(256), 0, s, (__bf16*)a, rows, n, ld);
  else hipLaunchKernelGGL(k_relu<float>, dim3(grid), dim3(256), 0, s, (float*)a, rows, n, ld);
  SPMM_HIP(hipGetLastError());
  return SPMM_OK;
}

// First-fit allocator over [0, size) in 256-byte units, with coalescing.
class Pool {
 public:
  explicit Pool(int64_t size) : size_(size) {
    if (size > 0) free_[0] = size;
  }
  // returns the offset, or -1 if no free range is large enough
  int64_t alloc(int64_t bytes) {
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const int64_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_ += bytes;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off, int64_t bytes) {
    bytes = round(bytes);
    used_ -= bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
  int64_t used() const { return used_; }
  static int64_t round(int64_t b) { return (b + 255) / 256 * 256; }

 private:
  int64_t size_;
  int64_t used_ = 0;
  std::map<int64_t, int64_t> free_;
};

struct Request {
  uint64_t id = 0;
  int64_t n = 0, ld = 0;
  const void* x_host = nullptr;
  void* y_host = nullptr;
  int64_t ld_host = 0;
  double submit_s = 0, admit_s = 0;
  int layer = 0;
  int64_t off = -1, bytes = 0;  // pool range: buffer 0 at off, buffer 1 after it
};

}  // namespace

struct spmm_srv_s {
  std::vector<const spmm_plan_s*> plans;
  std::vector<int64_t> dims;
  std::vector<uint8_t> relu;
  int L = 0;
  spmm_serve_opts opts{};
  spmm_dtype_t act = SPMM_F16;  // activation dtype (x of layer 0, y of every layer)
  int elem = 2;
  int64_t side0 = 0, side1 = 0;  // rows of ping-pong buffers 0 and 1
  int device = 0;

  std::mutex mu;
  std::condition_variable cv;       // wakes the worker (submit, stop)
  std::condition_variable done_cv;  // wakes drain
  std::deque<Request> pending;
  std::vector<Request> active;
  std::deque<spmm_serve_done_t> done;
  int64_t outstanding = 0;          // submitted and not yet done
  spmm_status_t failed = SPMM_OK;
  std::string fail_msg;
  bool stop = false;
  std::thread worker;

  Pool* pool = nullptr;
  uint8_t* pool_dev = nullptr;
  hipStream_t stream = nullptr;       // the layers' kernels
  hipStream_t up_stream = nullptr;    // request inputs over PCIe, overlapping earlier steps' kernels
  hipStream_t down_stream = nullptr;  // request outputs over PCIe, after their step's kernels
  hipEvent_t up_ev = nullptr;         // a step's uploads done (the kernels wait for it)
  hipEvent_t done_ev = nullptr;       // a step's kernels done (the downloads wait for it)
  spmm_group_t group = nullptr;
  spmm_serve_stats_t stats{};

  // steps enqueued on the device and not yet retired (worker mode): the event
  // recorded after the step and the requests whose output it copies back
  struct InFlight {
    hipEvent_t ev = nullptr;
    std::vector<Request> finished;
  };
  std::deque<InFlight> inflight;
  std::vector<hipEvent_t> free_events;
  int64_t active_tokens = 0;        // sum of n over `active`

  // scratch for grouped runs
  std::vector<spmm_plan_t> g_plans;
  std::vector<int64_t> g_n, g_ldx, g_ldy;
  std::vector<const void*> g_x;
  std::vector<void*> g_y;
  std::vector<uint8_t> g_relu;
};

static int64_t request_bytes(const spmm_srv_s* s, int64_t n) {
  const int64_t ld = (n + 7) / 8 * 8;
  return Pool::round(s->side0 * ld * s->elem) + Pool::round(s->side1 * ld * s->elem);
}

static void* buffer(spmm_srv_s* s, const Request& r, int which) {
  if (s->opts.simulate) return nullptr;
  uint8_t* base = s->pool_dev + r.off;
  return which == 0 ? (void*)base : (void*)(base + Pool::round(s->side0 * r.ld * s->elem));
}

// Admission from the FIFO head (caller holds mu). Returns the admitted requests.
// A request waits while the slots, the pool or the per-step token budget
// (tokens of all admitted requests; a lone request is always admitted) is
// exhausted; later requests wait behind it.
static std::vector<Request> admit_locked(spmm_srv_s* s, int limit) {
  std::vector<Request> out;
  int64_t tokens = s->active_tokens;
  while (!s->pending.empty() && (int)(s->active.size() + out.size()) < limit) {
    Request& r = s->pending.front();
    const bool alone = s->active.empty() && out.empty();
    if (s->opts.max_tokens > 0 && !alone && tokens + r.n > s->opts.max_tokens) break;
    const int64_t off = s->pool->alloc(r.bytes);
    if (off < 0) break;  // head-of-line: later requests wait for the head
    r.off = off;
    r.admit_s = now_s();
    tokens += r.n;
    out.push_back(r);
    s->pending.pop_front();
  }
  return out;
}

// Host <-> device copies of a request's input and output: one contiguous copy
// when the host layout equals the device layout, else a strided one. Uploads
// run on a stream of their own that waits for nothing, so they overlap the
// kernels of the steps before; a step's kernels wait for its uploads (up_ev).
// Downloads run on a second stream after the step's kernels (done_ev), and the
// step's completion event is recorded there, so a request's memory returns to
// the pool only once its output has left the device. Memory that an upload
// writes was released by an earlier completion event, which follows every
// kernel of its step and of the steps before it.
static spmm_status_t upload_input(spmm_srv_s* s, const Request& r) {
  if (s->opts.simulate) return SPMM_OK;
  if (r.ld_host == r.ld)
    SPMM_HIP(hipMemcpyAsync(buffer(s, r, 0), r.x_host, (size_t)(s->dims[0] * r.ld * s->elem), hipMemcpyHostToDevice,
                            s->up_stream));
  else
    SPMM_HIP(hipMemcpy2DAsync(buffer(s, r, 0), (size_t)(r.ld * s->elem), r.x_host, (size_t)(r.ld_host * s->elem),
                              (size_t)(r.n * s->elem), (size_t)s->dims[0], hipMemcpyHostToDevice, s->up_stream));
  return SPMM_OK;
}

static spmm_status_t download_output(spmm_srv_s* s, const Request& r) {
  if (s->opts.simulate) return SPMM_OK;
  if (r.ld_host == r.ld)
    SPMM_HIP(hipMemcpyAsync(r.y_host, buffer(s, r, s->L % 2), (size_t)(s->dims[s->L] * r.ld * s->elem),
                            hipMemcpyDeviceToHost, s->down_stream));
  else
    SPMM_HIP(hipMemcpy2DAsync(r.y_host, (size_t)(r.ld_host * s->elem), buffer(s, r, s->L % 2),
                              (size_t)(r.ld * s->elem), (size_t)(r.n * s->elem), (size_t)s->dims[s->L],
                              hipMemcpyDeviceToHost, s->down_stream));
  return SPMM_OK;
}

static void finish_locked(spmm_srv_s* s, const Request& r, double t) {
  s->pool->release(r.off, r.bytes);
  spmm_serve_done_t d;
  d.id = r.id;
  d.n = r.n;
  d.submit_s = r.submit_s;
  d.admit_s = r.admit_s;
  d.done_s = t;
  s->done.push_back(d);
  s->stats.requests_done += 1;
  s->stats.tokens_done += r.n;
  s->outstanding -= 1;
}

// Retires enqueued steps whose event has completed (all of them when `wait`):
// their finished requests release their memory and are reported done.
static spmm_status_t retire(spmm_srv_s* s, bool wait_all, bool wait_one) {
  spmm_status_t st = SPMM_OK;
  while (!s->inflight.empty()) {
    spmm_srv_s::InFlight& f = s->inflight.front();
    hipError_t e = hipEventQuery(f.ev);
    if (e == hipErrorNotReady) {
      if (!wait_all && !wait_one) break;
      e = hipEventSynchronize(f.ev);
      wait_one = false;
    }
    if (e != hipSuccess) {
      st = fail_hip(e, "serving step");
      break;
    }
    const double t = now_s();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      for (const Request& r : f.finished) finish_locked(s, r, t);
    }
    s->free_events.push_back(f.ev);
    s->inflight.pop_front();
    s->done_cv.notify_all();
  }
  return st;
}

// One step. Manual and simulated servers complete each step before returning
// (requests finishing in it are done on return); the worker enqueues steps and
// retires them as their events complete, at most two steps ahead of the device.
static spmm_status_t do_step(spmm_srv_s* s, int32_t* remaining) {
  const double t0 = now_s();
  const bool async = !s->opts.manual && !s->opts.simulate && s->opts.mode == SPMM_SERVE_CONTINUOUS;
  spmm_status_t st = SPMM_OK;
  if (async) st = retire(s, false, s->inflight.size() >= 2);
  std::vector<Request> admitted;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->failed != SPMM_OK) return s->failed;
    if (st == SPMM_OK) admitted = admit_locked(s, s->opts.mode == SPMM_SERVE_PLAIN ? 1 : s->opts.max_active);
  }
  for (const Request& r : admitted)
    if (st == SPMM_OK) st = upload_input(s, r);
  if (st == SPMM_OK && !admitted.empty() && !s->opts.simulate) {
    hipError_t e = hipEventRecord(s->up_ev, s->up_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(s->stream, s->up_ev, 0);
    if (e != hipSuccess) st = fail_hip(e, "upload fence");
  }
  for (Request& r : admitted) {  // only the stepping thread touches `active`
    s->active.push_back(r);
    s->active_tokens += r.n;
  }
  // statistics are read by spmm_serve_stats on other threads: every update
  // holds mu (here, and the counts below in the closing lock)
  int64_t problems = 0, steps = 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stats.peak_pool_bytes = std::max(s->stats.peak_pool_bytes, s->pool->used());
    s->stats.peak_active = std::max(s->stats.peak_active, (int32_t)s->active.size());
  }

  std::vector<Request> finished;
  if (st == SPMM_OK && !s->active.empty()) {
    if (s->opts.mode == SPMM_SERVE_PLAIN) {
      // the one admitted request, every layer with its own launches
      Request& r = s->active.front();
      for (int l = 0; l < s->L && st == SPMM_OK; ++l) {
        if (!s->opts.simulate) {
          void* X = buffer(s, r, l % 2);
          void* Y = buffer(s, r, (l + 1) % 2);
          st = run_plan(s->plans[l], r.n, X, r.ld, Y, r.ld, plan_variant(s->plans[l], r.n), false, s->stream);
          if (st == SPMM_OK && s->relu[l]) st = launch_relu(s->act, Y, s->dims[l + 1], r.n, r.ld, s->stream);
        }
        problems += 1;
      }
      r.layer = s->L;
    } else {
      const size_t cnt = s->active.size();
      s->g_plans.resize(cnt);
      s->g_n.resize(cnt);
      s->g_ldx.resize(cnt);
      s->g_ldy.resize(cnt);
      s->g_x.resize(cnt);
      s->g_y.resize(cnt);
      s->g_relu.resize(cnt);
      for (size_t i = 0; i < cnt; ++i) {
        const Request& r = s->active[i];
        s->g_plans[i] = s->opts.simulate ? nullptr : const_cast<spmm_plan_s*>(s->plans[r.layer]);
        s->g_n[i] = r.n;
        s->g_ldx[i] = r.ld;
        s->g_ldy[i] = r.ld;
        s->g_x[i] = buffer(s, r, r.layer % 2);
        s->g_y[i] = buffer(s, r, (r.layer + 1) % 2);
        s->g_relu[i] = s->relu[r.layer];
      }
      if (!s->opts.simulate)
        st = spmm_group_run(s->group, (int32_t)cnt, s->g_plans.data(), s->g_n.data(), s->g_x.data(), s->g_ldx.data(),
                            s->g_y.data(), s->g_ldy.data(), s->g_relu.data(), s->stream);
      problems += (int64_t)cnt;
      for (Request& r : s->active) r.layer += 1;
    }
    if (st == SPMM_OK && !s->opts.simulate) {
      hipError_t e = hipEventRecord(s->done_ev, s->stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(s->down_stream, s->done_ev, 0);
      if (e != hipSuccess) st = fail_hip(e, "step fence");
    }
    for (const Request& r : s->active)
      if (r.layer == s->L && st == SPMM_OK) st = download_output(s, r);
    size_t w = 0;
    for (size_t i = 0; i < s->active.size(); ++i) {
      if (s->active[i].layer == s->L) {
        finished.push_back(s->active[i]);
        s->active_tokens -= s->active[i].n;
      } else {
        s->active[w++] = s->active[i];
      }
    }
    s->active.resize(w);
    steps += 1;
    if (st == SPMM_OK && async) {
      spmm_srv_s::InFlight f;
      if (!s->free_events.empty()) {
        f.ev = s->free_events.back();
        s->free_events.pop_back();
      } else {
        hipError_t e = hipEventCreateWithFlags(&f.ev, hipEventDisableTiming);
        if (e != hipSuccess) st = fail_hip(e, "hipEventCreate");
      }
      if (st == SPMM_OK) {
        hipError_t e = hipEventRecord(f.ev, s->down_stream);  // after the step's kernels and downloads
        if (e != hipSuccess) st = fail_hip(e, "hipEventRecord");
      }
      if (st == SPMM_OK) {
        f.finished.swap(finished);
        s->inflight.push_back(std::move(f));
      } else if (f.ev) {
        s->free_events.push_back(f.ev);
      }
    } else if (st == SPMM_OK && !s->opts.simulate) {
      hipError_t e = hipStreamSynchronize(s->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->down_stream);
      if (e != hipSuccess) st = fail_hip(e, "serving step");
    }
  } else if (st == SPMM_OK && async && !s->inflight.empty()) {
    st = retire(s, false, true);  // nothing to enqueue: wait for the oldest step
  }
  const double t1 = now_s();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (st != SPMM_OK) {
      s->failed = st;
      s->fail_msg = spmm_last_error();
    }
    for (const Request& r : finished) finish_locked(s, r, t1);
    s->stats.problems_run += problems;
    s->stats.steps += steps;
    s->stats.busy_s += t1 - t0;
    if (remaining) *remaining = (int32_t)(s->pending.size() + s->active.size() + s->inflight.size());
  }
  s->done_cv.notify_all();
  return st;
}

static void worker_main(spmm_srv_s* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [&] { return s->stop || !s->pending.empty() || !s->active.empty() || !s->inflight.empty(); });
      if (s->stop) return;
      if (s->failed != SPMM_OK) {
        s->done_cv.notify_all();
        s->cv.wait(lk, [&] { return s->stop; });
        return;
      }
    }
    int32_t rem = 0;
    (void)do_step(s, &rem);
  }
}

static void destroy_server(spmm_srv_s* s) {
  if (s->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv.notify_all();
    s->worker.join();
  }
  if (s->stream) {
    (void)hipStreamSynchronize(s->stream);
    (void)hipStreamDestroy(s->stream);
  }
  for (hipStream_t cs : {s->up_stream, s->down_stream}) {
    if (cs) {
      (void)hipStreamSynchronize(cs);
      (void)hipStreamDestroy(cs);
    }
  }
  if (s->up_ev) (void)hipEventDestroy(s->up_ev);
  if (s->done_ev) (void)hipEventDestroy(s->done_ev);
  for (auto& f : s->inflight) (void)hipEventDestroy(f.ev);
  for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
  if (s->group) (void)spmm_group_destroy(s->group);
  if (s->pool_dev) (void)hipFree(s->pool_dev);
  delete s->pool;
  delete s;
}

extern "C" {

double spmm_serve_clock(void) { return now_s(); }

spmm_status_t spmm_serve_create(const spmm_plan_t* layer_plans, int32_t num_layers, const int64_t* dims,
                                const uint8_t* relu_after, const spmm_serve_opts* opts, spmm_srv_t* out) {
  clear_error();
  if (!out) return fail(SPMM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!opts) return fail(SPMM_ERR_INVALID_ARG, "opts is NULL");
  if (num_layers < 1 || num_layers > 4096) return fail(SPMM_ERR_INVALID_ARG, "num_layers must be in [1, 4096]");
  if (!dims) return fail(SPMM_ERR_INVALID_ARG, "dims is NULL");
  if (opts->mode != SPMM_SERVE_CONTINUOUS && opts->mode != SPMM_SERVE_PLAIN)
    return fail(SPMM_ERR_INVALID_ARG, "unknown serving mode");
  if (opts->mem_budget_bytes <= 0) return fail(SPMM_ERR_INVALID_ARG, "mem_budget_bytes must be positive");
  if (opts->max_active < 1 || opts->max_active > 65536) return fail(SPMM_ERR_INVALID_ARG, "max_active must be in [1, 65536]");
  for (int l = 0; l <= num_layers; ++l)
    if (dims[l] < 1) return fail(SPMM_ERR_INVALID_ARG, "feature sizes must be positive");
  if (!opts->simulate) {
    if (!layer_plans) return fail(SPMM_ERR_INVALID_ARG, "layer_plans is NULL");
    for (int l = 0; l < num_layers; ++l) {
      const spmm_plan_s* p = layer_plans[l];
      if (!p) return fail(SPMM_ERR_INVALID_ARG, "a layer plan is NULL");
      if (!p->has_values) return fail(SPMM_ERR_INVALID_ARG, "values were not set on a layer plan");
      if (p->k != dims[l] || p->m != dims[l + 1]) return fail(SPMM_ERR_INVALID_ARG, "plan shapes do not match dims");
      if (l > 0 && layer_plans[l - 1]->y != p->x)
        return fail(SPMM_ERR_INVALID_ARG, "output dtype of a layer differs from the next layer's input dtype");
      if (p->y != layer_plans[0]->x) return fail(SPMM_ERR_INVALID_ARG, "all activations must share one dtype");
    }
  }
  spmm_srv_s* s = new (std::nothrow) spmm_srv_s;
  if (!s) return fail(SPMM_ERR_OOM, "host allocation failed");
  s->L = num_layers;
  s->opts = *opts;
  s->dims.assign(dims, dims + num_layers + 1);
  s->relu.assign(num_layers, 0);
  if (relu_after)
    for (int l = 0; l < num_layers; ++l) s->relu[l] = relu_after[l] ? 1 : 0;
  if (!opts->simulate) {
    s->plans.assign(layer_plans, layer_plans + num_layers);
    s->act = s->plans[0]->x;
    s->elem = dtype_bytes(s->act);
  }
  // buffer 0 holds the inputs of even layers and outputs of odd ones; buffer 1 the rest
  for (int l = 0; l < num_layers; ++l) {
    int64_t& in_side = (l % 2 == 0) ? s->side0 : s->side1;
    int64_t& out_side = (l % 2 == 0) ? s->side1 : s->side0;
    in_side = std::max(in_side, dims[l]);
    out_side = std::max(out_side, dims[l + 1]);
  }
  s->pool = new (std::nothrow) Pool(opts->mem_budget_bytes);
  spmm_status_t st = s->pool ? SPMM_OK : fail(SPMM_ERR_OOM, "host allocation failed");
  if (st == SPMM_OK && !opts->simulate) {
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) st = fail_hip(e, "hipGetDevice");
    if (st == SPMM_OK && (e = hipMalloc((void**)&s->pool_dev, (size_t)opts->mem_budget_bytes)) != hipSuccess)
      st = fail_hip(e, "hipMalloc activation pool");
    if (st == SPMM_OK && (e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking)) != hipSuccess)
      st = fail_hip(e, "hipStreamCreate");
    if (st == SPMM_OK && (e = hipStreamCreateWithFlags(&s->up_stream, hipStreamNonBlocking)) != hipSuccess)
      st = fail_hip(e, "hipStreamCreate");
    if (st == SPMM_OK && (e = hipStreamCreateWithFlags(&s->down_stream, hipStreamNonBlocking)) != hipSuccess)
      st = fail_hip(e, "hipStreamCreate");
    if (st == SPMM_OK && (e = hipEventCreateWithFlags(&s->up_ev, hipEventDisableTiming)) != hipSuccess)
      st = fail_hip(e, "hipEventCreate");
    if (st == SPMM_OK && (e = hipEventCreateWithFlags(&s->done_ev, hipEventDisableTiming)) != hipSuccess)
      st = fail_hip(e, "hipEventCreate");
    if (st == SPMM_OK && opts->mode == SPMM_SERVE_CONTINUOUS) {
      for (int l = 0; l < num_layers && st == SPMM_OK; ++l)
        if (!plan_uses_row_kernel(s->plans[l]) || s->plans[l]->w == SPMM_FP8_E4M3 || s->plans[l]->b > 32 ||
            s->plans[l]->b != s->plans[0]->b || s->plans[l]->w != s->plans[0]->w || s->plans[l]->y != s->plans[0]->y)
          st = fail(SPMM_ERR_UNSUPPORTED,
                    "continuous batching needs layers of one block size (16 or 32) and one 16-bit dtype");
      if (st == SPMM_OK) st = spmm_group_create(opts->max_active, &s->group);
    }
  }
  if (st == SPMM_OK && !opts->manual) {
    try {
      s->worker = std::thread(worker_main, s);
    } catch (...) {
      st = fail(SPMM_ERR_OOM, "could not start the serving thread");
    }
  }
  if (st != SPMM_OK) {
    destroy_server(s);
    return st;
  }
  *out = s;
  return SPMM_OK;
}

spmm_status_t spmm_serve_submit(spmm_srv_t s, uint64_t id, int64_t n, const void* x_host, void* y_host,
                                int64_t ld_host) {
  clear_error();
  if (!s) return fail(SPMM_ERR_INVALID_ARG, "server is NULL");
  if (n < 1 || n > (1 << 24)) return fail(SPMM_ERR_INVALID_ARG, "n must be in [1, 2^24]");
  if (ld_host < n) return fail(SPMM_ERR_INVALID_ARG, "ld_host is smaller than n");
  if (!s->opts.simulate && (!x_host || !y_host)) return fail(SPMM_ERR_INVALID_ARG, "x_host and y_host are required");
  Request r;
  r.id = id;
  r.n = n;
  r.ld = (n + 7) / 8 * 8;
  r.x_host = x_host;
  r.y_host = y_host;
  r.ld_host = ld_host;
  r.bytes = request_bytes(s, n);
  if (r.bytes > s->opts.mem_budget_bytes) return fail(SPMM_ERR_REJECTED, "request exceeds the activation memory budget");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->failed != SPMM_OK) return fail(s->failed, s->fail_msg);
    r.submit_s = now_s();
    s->pending.push_back(r);
    s->outstanding += 1;
  }
  s->cv.notify_one();
  return SPMM_OK;
}

spmm_status_t spmm_serve_poll(spmm_srv_t s, spmm_serve_done_t* out, int32_t max, int32_t* num_done) {
  clear_error();
  if (!s || !num_done) return fail(SPMM_ERR_INVALID_ARG, "server or num_done is NULL");
  if (max > 0 && !out) return fail(SPMM_ERR_INVALID_ARG, "out is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  int32_t k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *num_done = k;
  return SPMM_OK;
}

spmm_status_t spmm_serve_step(spmm_srv_t s, int32_t* active_out) {
  clear_error();
  if (!s) return fail(SPMM_ERR_INVALID_ARG, "server is NULL");
  if (!s->opts.manual) return fail(SPMM_ERR_INVALID_ARG, "spmm_serve_step is for manual servers");
  return do_step(s, active_out);
}

spmm_status_t spmm_serve_drain(spmm_srv_t s) {
  clear_error();
  if (!s) return fail(SPMM_ERR_INVALID_ARG, "server is NULL");
  if (s->opts.manual) {
    int32_t rem = 1;
    while (rem > 0) {
      spmm_status_t st = do_step(s, &rem);
      if (st != SPMM_OK) return st;
    }
    return SPMM_OK;
  }
  std::unique_lock<std::mutex> lk(s->mu);
  s->done_cv.wait(lk, [&] { return s->outstanding == 0 || s->failed != SPMM_OK; });
  if (s->failed != SPMM_OK) return fail(s->failed, s->fail_msg);
  return SPMM_OK;
}

spmm_status_t spmm_serve_stats(spmm_srv_t s, spmm_serve_stats_t* out) {
  clear_error();
  if (!s || !out) return fail(SPMM_ERR_INVALID_ARG, "server or out is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->pending = (int32_t)s->pending.size();
  out->active = (int32_t)(s->outstanding - (int64_t)s->pending.size());
  return SPMM_OK;
}

spmm_status_t spmm_serve_destroy(spmm_srv_t s) {
  clear_error();
  if (!s) return SPMM_OK;
  destroy_server(s);
  return SPMM_OK;
}

}  // extern "C"
