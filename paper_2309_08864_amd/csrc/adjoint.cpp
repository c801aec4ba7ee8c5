// adjoint.cpp -- reverse-mode gradient of the sweep (not yet built).
#include "plan.hpp"

namespace so2dr {

int adjoint_run(Plan &P, const void *, const void *, void *, double *, double *, int,
                void *const *, int, so2dr_stats *) {
  (void)P;
  set_error("adjoint not built in this library version");
  return SO2DR_E_UNSUPPORTED;
}

}  // namespace so2dr
