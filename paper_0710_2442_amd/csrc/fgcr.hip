// Flexible GCR with a right preconditioner (placeholder until the network lands).
#include "wd_solver.h"

namespace wd {

wd_status solve_fgcr(wd_gauge *, const void *, void *, double, double, const wd_solve_params &, wd_solve_info &,
                     hipStream_t) {
  return set_error(WD_ERR_ARG, "FGCR solver is not available in this build");
}

void ptc_release(wd_gauge *) {}

}  // namespace wd
