// Entry points whose implementation is not built yet.
#include "internal.h"

extern "C" {
hpeps_status hpeps_peps_energy(hpeps_ctx*, const hpeps_peps*, int32_t, const int32_t*, const int32_t*,
                               const double*, const int64_t*, const hpeps_esvd_opts*, double*, double*) {
  return HPEPS_ERR_UNSUPPORTED;
}
hpeps_status hpeps_apply_two_site_gate(hpeps_ctx*, hpeps_peps*, const int64_t*, int32_t, int32_t, int32_t,
                                       const void*, int64_t, int64_t*, double*) {
  return HPEPS_ERR_UNSUPPORTED;
}
hpeps_status hpeps_ite_plan_create(hpeps_ctx*, const hpeps_peps*, int32_t, const void*, const int32_t*,
                                   int64_t, hpeps_ite_plan**) {
  return HPEPS_ERR_UNSUPPORTED;
}
hpeps_status hpeps_ite_run(hpeps_ite_plan*, int32_t, int32_t) { return HPEPS_ERR_UNSUPPORTED; }
hpeps_status hpeps_ite_get_state(hpeps_ite_plan*, int64_t*, void* const*) { return HPEPS_ERR_UNSUPPORTED; }
hpeps_status hpeps_ite_plan_destroy(hpeps_ite_plan*) { return HPEPS_ERR_UNSUPPORTED; }
}
