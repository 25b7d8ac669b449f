// Entry points whose kernels are not built yet.
#include "handle.hpp"

extern "C" {
sislice_status sislice_plan_shifts_kpm(sislice_handle*, int64_t, const double*, int64_t,
                                       const double*, int64_t, int64_t, int64_t,
                                       const sislice_opts*, double*, double*, double*, double*) {
  return SISLICE_ERR_ARG;
}
sislice_status sislice_solve(sislice_handle*, int64_t, const double*, int64_t, const double*,
                             int64_t, int64_t, int64_t, const double*, double*, const sislice_opts*,
                             double*, double*, int64_t, double*, sislice_report*) {
  return SISLICE_ERR_ARG;
}

}
