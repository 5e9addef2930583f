// Block sizes 1, 4 and 8 (placeholder until the small-block kernel lands).
#include "common.h"

namespace spmm {
spmm_status_t launch_spmm_small(const RunArgs& a, hipStream_t s) {
  (void)a;
  (void)s;
  return fail(SPMM_ERR_UNSUPPORTED, "block sizes 1, 4 and 8 are not built yet");
}
}  // namespace spmm
