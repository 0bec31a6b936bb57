// cbase.hip -- placeholder for the complex-arithmetic baselines.
#include "../../include/frobinv.h"
extern "C" {
frob_status_t frob_cinv_lu(frob_handle_t, int, const double*, const double*, int, double*, double*, int, int,
                           frob_result_t*) {
  return FROB_E_INTERNAL;
}
frob_status_t frob_cinv_chol(frob_handle_t, int, const double*, const double*, int, double*, double*, int, int,
                             frob_result_t*) {
  return FROB_E_INTERNAL;
}
}
