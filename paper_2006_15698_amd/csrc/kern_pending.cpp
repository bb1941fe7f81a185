// Entry points whose kernels are not built yet: they report
// hipErrorNotSupported so that the C ABI returns DG_EHIP / DG_EUNSUPPORTED.
#include "dg_internal.h"

bool dg_f32_supported(int) { return false; }
int dg_launch_rhs_f32(const dg_ctx*, const double*, const double*, double*) { return (int)hipErrorNotSupported; }
int dg_launch_stage_f32(const dg_ctx*, double*, double*, const double*, double*, double, double, double, int) {
  return (int)hipErrorNotSupported;
}
int dg_launch_vjp(const dg_ctx*, const double*, const double*, double*, char*) { return (int)hipErrorNotSupported; }
