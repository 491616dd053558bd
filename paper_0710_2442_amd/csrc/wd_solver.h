// Host-side solver entry points (called by the C-ABI layer).
#pragma once

#include "wd_internal.h"

namespace wd {

wd_status solve(wd_gauge *g, const void *b, void *x, double kappa, double tol, const wd_solve_params &prm,
                wd_solve_info &info);
wd_status solve_mrhs(wd_gauge *g, const void *b, void *x, int nrhs, double kappa, double tol,
                     const wd_solve_params &prm, wd_solve_info *infos);
wd_status solve_fgcr(wd_gauge *g, const void *b, void *x, double kappa, double tol, const wd_solve_params &prm,
                     wd_solve_info &info, hipStream_t st);
void workspace_free(wd_gauge *g);
// release the mixed FGCR's cached buffers (fgcr.hip)
void fgcr_free(wd_gauge *g);
wd_status solve_batch(const wd_gauge *const *gs, int n, const void *const *b, void *const *x, const double *kappa,
                      double tol, const wd_solve_params &prm, wd_solve_info *infos);
// FP64 defect correction around an FP32 even-odd FGCR(m) with the network
// (or the identity) as right preconditioner
wd_status solve_fgcr_mixed(wd_gauge *g, const void *b, void *x, double kappa, double tol, const wd_solve_params &prm,
                           wd_solve_info &info, hipStream_t st);
struct CgScalars;
// r = b - D_W x in FP64 (nsys systems sys_stride bytes apart), |r|^2 -> sc[y].rnorm2
wd_status true_residual64(const wd_gauge *g, const void *b, const void *x, void *r, int nsys, size_t sys_stride,
                          double kappa, CgScalars *sc, RedBuf red, hipStream_t st);
// FP64 even-odd CGLS on stream st (synchronises st)
wd_status solve_cg64(wd_gauge *g, const void *b, void *x, double kappa, double tol, const wd_solve_params &prm,
                     wd_solve_info &info, hipStream_t st);

}  // namespace wd

namespace wd {
// release the PTC preconditioner state a handle may hold (ptc.hip)
void ptc_release(wd_gauge *g);
}  // namespace wd
