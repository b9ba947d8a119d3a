// Placeholder until the compensated-FP32 kernels land.
#include "frg_ctx.h"

namespace frg {
int Context::integrate_fp32c_sets(const std::vector<SetDev> &, int, hipStream_t) {
  return fail(FRG_E_INVAL, "FRG_PREC_FP32C is not available in this build");
}
int Context::grid_fp32c(const frg_quad &, int64_t, const double *, int64_t, const double *,
                        double *, double *, uint8_t *, hipStream_t) {
  return fail(FRG_E_INVAL, "FRG_PREC_FP32C is not available in this build");
}
}  // namespace frg
