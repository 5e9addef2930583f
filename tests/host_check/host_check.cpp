// Host-side checks of the library under AddressSanitizer and
// UndefinedBehaviorSanitizer (the library's host code is built with both, its
// GPU code as usual). Everything here runs without a GPU: the serving
// scheduler in simulate mode, and the argument validation of the C ABI that
// rejects bad input before any device work. Exits non-zero on the first
// unexpected result; a sanitizer finding aborts the process.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "../../include/spmm.h"

static int failures = 0;
#define CHECK(cond)                                                    \
  do {                                                                 \
    if (!(cond)) {                                                     \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                      \
    }                                                                  \
  } while (0)

static void serve_simulated(int mode, bool manual, int64_t max_tokens, uint32_t seed) {
  const int32_t layers = 4;
  const int64_t dims[layers + 1] = {256, 1024, 256, 1024, 256};
  const uint8_t relu[layers] = {1, 0, 1, 0};
  spmm_serve_opts opts;
  std::memset(&opts, 0, sizeof opts);
  opts.mem_budget_bytes = (int64_t)64 * (1024 + 256) * 2 * 8;  // room for a few requests
  opts.max_active = 7;
  opts.mode = mode;
  opts.manual = manual ? 1 : 0;
  opts.simulate = 1;
  opts.max_tokens = max_tokens;
  spmm_srv_t srv = nullptr;
  CHECK(spmm_serve_create(nullptr, layers, dims, relu, &opts, &srv) == SPMM_OK && srv);
  if (!srv) return;
  std::mt19937 g(seed);
  int64_t submitted = 0, tokens = 0;
  for (uint64_t id = 0; id < 300; ++id) {
    const int64_t n = 1 + (int64_t)(g() % 64);
    const spmm_status_t st = spmm_serve_submit(srv, id, n, nullptr, nullptr, n);
    CHECK(st == SPMM_OK);
    if (st == SPMM_OK) {
      ++submitted;
      tokens += n;
    }
    if (manual && id % 5 == 0) {
      int32_t active = -1;
      CHECK(spmm_serve_step(srv, &active) == SPMM_OK && active >= 0);
    }
  }
  // a request larger than the whole pool is refused
  CHECK(spmm_serve_submit(srv, 1000000, (int64_t)1 << 20, nullptr, nullptr, (int64_t)1 << 20) == SPMM_ERR_REJECTED);
  CHECK(spmm_serve_submit(srv, 1000001, 0, nullptr, nullptr, 1) == SPMM_ERR_INVALID_ARG);
  CHECK(spmm_serve_drain(srv) == SPMM_OK);
  std::vector<spmm_serve_done_t> done(64);
  int64_t got = 0, got_tokens = 0;
  std::vector<uint8_t> seen(300, 0);
  for (;;) {
    int32_t k = 0;
    CHECK(spmm_serve_poll(srv, done.data(), (int32_t)done.size(), &k) == SPMM_OK);
    if (k == 0) break;
    for (int32_t i = 0; i < k; ++i) {
      CHECK(done[i].id < 300 && !seen[done[i].id]);
      if (done[i].id < 300) seen[done[i].id] = 1;
      CHECK(done[i].submit_s <= done[i].admit_s && done[i].admit_s <= done[i].done_s);
      got_tokens += done[i].n;
    }
    got += k;
  }
  CHECK(got == submitted && got_tokens == tokens);
  spmm_serve_stats_t stats;
  CHECK(spmm_serve_stats(srv, &stats) == SPMM_OK);
  CHECK(stats.requests_done == submitted && stats.tokens_done == tokens && stats.pending == 0 && stats.active == 0);
  CHECK(stats.peak_pool_bytes <= opts.mem_budget_bytes);
  if (mode == SPMM_SERVE_CONTINUOUS) CHECK(stats.peak_active <= opts.max_active);
  CHECK(spmm_serve_destroy(srv) == SPMM_OK);
}

static void validation() {
  // ELL: index out of range, repeated column, bad width, NULL
  const int32_t bad_col[4] = {0, 9, -1, -1};
  const int32_t rep[4] = {1, 1, 0, -1};
  const int32_t ok_cols[4] = {0, 1, 1, -1};
  spmm_plan_t p = nullptr;
  CHECK(spmm_plan_ell(32, 32, 16, 2, bad_col, SPMM_F16, SPMM_F16, SPMM_F16, nullptr, &p) == SPMM_ERR_INVALID_ARG && !p);
  CHECK(spmm_plan_ell(32, 32, 16, 2, rep, SPMM_F16, SPMM_F16, SPMM_F16, nullptr, &p) == SPMM_ERR_INVALID_ARG && !p);
  CHECK(spmm_plan_ell(32, 32, 16, -1, ok_cols, SPMM_F16, SPMM_F16, SPMM_F16, nullptr, &p) == SPMM_ERR_INVALID_ARG);
  CHECK(spmm_plan_ell(32, 32, 16, 2, nullptr, SPMM_F16, SPMM_F16, SPMM_F16, nullptr, &p) == SPMM_ERR_INVALID_ARG);
  CHECK(std::strlen(spmm_last_error()) > 0);
  // static plans: block size, NULL mask, dtype triple, options
  std::vector<uint8_t> mask(64, 1);
  CHECK(spmm_plan_static(128, 128, 3, mask.data(), SPMM_F16, SPMM_F16, SPMM_F16, nullptr, &p) == SPMM_ERR_INVALID_ARG);
  CHECK(spmm_plan_static(128, 128, 16, nullptr, SPMM_F16, SPMM_F16, SPMM_F16, nullptr, &p) == SPMM_ERR_INVALID_ARG);
  CHECK(spmm_plan_static(0, 128, 16, mask.data(), SPMM_F16, SPMM_F16, SPMM_F16, nullptr, &p) == SPMM_ERR_INVALID_ARG);
  CHECK(spmm_plan_static(128, 128, 16, mask.data(), SPMM_FP8_E4M3, SPMM_F32, SPMM_F32, nullptr, &p) ==
        SPMM_ERR_UNSUPPORTED);
  spmm_plan_opts o;
  std::memset(&o, 0, sizeof o);
  o.variant = 3;
  CHECK(spmm_plan_static(128, 128, 16, mask.data(), SPMM_F16, SPMM_F16, SPMM_F16, &o, &p) == SPMM_ERR_INVALID_ARG);
  o.variant = 0;
  o.dense_dispatch = 7;
  CHECK(spmm_plan_static(128, 128, 16, mask.data(), SPMM_F16, SPMM_F16, SPMM_F16, &o, &p) == SPMM_ERR_INVALID_ARG);
  o.dense_dispatch = 0;
  o.variant = 3 * 256;
  CHECK(spmm_plan_static(128, 128, 16, mask.data(), SPMM_F16, SPMM_F16, SPMM_F16, &o, &p) == SPMM_ERR_INVALID_ARG);
  // speedup model over its domain and outside it
  double s = 0.0;
  for (int64_t m = 256; m <= 8192; m *= 2)
    for (int32_t b : {1, 4, 8, 16})
      for (double d : {1.0 / 32, 1.0 / 8, 1.0}) {
        CHECK(spmm_speedup_model(m, d, b, &s) == SPMM_OK && std::isfinite(s) && s > 0.0);
      }
  CHECK(spmm_speedup_model(0, 0.5, 16, &s) == SPMM_ERR_INVALID_ARG);
  CHECK(spmm_speedup_model(64, 1.5, 16, &s) == SPMM_ERR_INVALID_ARG);
  // NULL handles across the ABI
  spmm_group_t gr = nullptr;
  CHECK(spmm_group_create(0, &gr) == SPMM_ERR_INVALID_ARG);
  CHECK(spmm_group_run(nullptr, 1, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
        SPMM_ERR_INVALID_ARG);
  CHECK(spmm_run_static(nullptr, 8, nullptr, 8, nullptr, 8, nullptr) == SPMM_ERR_INVALID_ARG);
  CHECK(spmm_plan_dispatch(nullptr, nullptr, nullptr) == SPMM_ERR_INVALID_ARG);
  CHECK(spmm_autotune_clear() == SPMM_OK);
  int32_t v = 0;
  CHECK(spmm_plan_variant(nullptr, 8, &v) == SPMM_ERR_INVALID_ARG);
  // serving: bad dims, NULL plans outside simulation
  const int64_t dims[3] = {64, 128, 64};
  spmm_serve_opts so;
  std::memset(&so, 0, sizeof so);
  so.mem_budget_bytes = 1 << 20;
  so.max_active = 4;
  spmm_srv_t srv = nullptr;
  CHECK(spmm_serve_create(nullptr, 2, dims, nullptr, &so, &srv) == SPMM_ERR_INVALID_ARG && !srv);
  so.simulate = 1;
  CHECK(spmm_serve_create(nullptr, 2, nullptr, nullptr, &so, &srv) == SPMM_ERR_INVALID_ARG && !srv);
}

int main() {
  validation();
  uint32_t seed = 1;
  for (int mode : {SPMM_SERVE_CONTINUOUS, SPMM_SERVE_PLAIN})
    for (bool manual : {true, false})
      for (int64_t max_tokens : {(int64_t)0, (int64_t)96}) serve_simulated(mode, manual, max_tokens, seed++);
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("host checks passed\n");
  return 0;
}
