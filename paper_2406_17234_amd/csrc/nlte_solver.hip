// JFNK solver (Algorithm 2) on the device.
#include "nlte_internal.h"

nlte_status set_err(nlte_status st, const char* fmt, ...);

extern "C" nlte_status nlte_zero_radiation_populations(nlte_column*, double*, hipStream_t) {
  return set_err(NLTE_E_INVALID, "not built yet");
}
extern "C" nlte_status nlte_solve(nlte_column*, const double*, const nlte_solve_opts*, double*,
                                  double*, nlte_solve_stats*, hipStream_t) {
  return set_err(NLTE_E_INVALID, "not built yet");
}
extern "C" nlte_status nlte_solve_batch(nlte_ctx*, nlte_column* const*, int32_t, const double* const*,
                                        const nlte_solve_opts*, double* const*, nlte_solve_stats*,
                                        hipStream_t) {
  return set_err(NLTE_E_INVALID, "not built yet");
}
