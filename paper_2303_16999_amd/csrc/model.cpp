// Power-law speedup model (C ABI): the paper's summary of its static sweep
// (Section 5) refitted to this library's static kernels against dense FP16
// GEMM on one MI355X.
#include <cmath>

#include "internal.h"

using namespace spmm;

namespace {
// Least-squares fit of log(speedup) over the grid m = k in 2^8 .. 2^13,
// b in {1, 4, 8, 16}, d in {1/4, 1/8, 1/16, 1/32}, FP16, sparse and dense each
// best over n in 4^1 .. 4^8 (96 points, R^2 = 0.909, rms error of log speedup
// 0.29).
constexpr double kA = 0.07649, kAlpha = -0.04109, kBeta = -0.6541, kGamma = 0.7269;
}  // namespace

extern "C" {

spmm_status_t spmm_speedup_model(int64_t m, double density, int32_t b, double* speedup) {
  clear_error();
  if (!speedup) return fail(SPMM_ERR_INVALID_ARG, "speedup is NULL");
  if (m < 1 || b < 1 || !(density > 0.0) || density > 1.0)
    return fail(SPMM_ERR_INVALID_ARG, "needs m >= 1, b >= 1 and 0 < density <= 1");
  *speedup = kA * std::pow((double)m, kAlpha) * std::pow(density, kBeta) * std::pow((double)b, kGamma);
  return SPMM_OK;
}

}  // extern "C"
