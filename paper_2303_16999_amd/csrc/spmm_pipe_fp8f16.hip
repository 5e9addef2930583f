// Instantiations of the pipelined SpMM kernel for X = _Float16, weights = Fp8.
#include "spmm_pipe.h"

namespace spmm {
namespace pipe {

template <typename YT>
static spmm_status_t dispatch_y(const RunArgs& a, hipStream_t s) {
  const int b = a.plan.b, rw = a.plan.group_rows / 8, nwv = a.pipe_nwv, ns = a.pipe_ns;
#define SPMM_V(B_, RW_, NS_, NWV_) \
  if (b == B_ && rw == RW_ && ns == NS_ && nwv == NWV_) return launch_pipe<_Float16, Fp8, YT, B_, RW_, NS_, NWV_>(a, s);
  SPMM_V(16, 4, 8, 4) SPMM_V(16, 4, 8, 8) SPMM_V(16, 2, 8, 4) SPMM_V(16, 2, 8, 8) SPMM_V(16, 1, 8, 8)
  SPMM_V(16, 4, 4, 4) SPMM_V(16, 4, 4, 8) SPMM_V(16, 2, 4, 4) SPMM_V(16, 2, 4, 8) SPMM_V(16, 1, 4, 8)
  SPMM_V(32, 2, 8, 4) SPMM_V(32, 2, 8, 8) SPMM_V(32, 1, 8, 8)
  SPMM_V(32, 2, 4, 4) SPMM_V(32, 2, 4, 8) SPMM_V(32, 1, 4, 8)
#undef SPMM_V
  return fail(SPMM_ERR_UNSUPPORTED, "no pipelined kernel variant for this geometry");
}

}  // namespace pipe

spmm_status_t launch_pipe_fp8f16(const RunArgs& a, hipStream_t s) {
  if (a.yt == SPMM_F32) return pipe::dispatch_y<float>(a, s);
  return pipe::dispatch_y<_Float16>(a, s);
}

}  // namespace spmm
