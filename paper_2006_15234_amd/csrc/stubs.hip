// Entry points whose implementation is not built yet.
#include "internal.h"

extern "C" {
hpeps_status hpeps_peps_energy(hpeps_ctx*, const hpeps_peps*, int32_t, const int32_t*, const int32_t*,
                               const double*, const int64_t*, const hpeps_esvd_opts*, double*, double*) {
  return HPEPS_ERR_UNSUPPORTED;
}
}
