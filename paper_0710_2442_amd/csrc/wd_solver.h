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
// Device buffers of a solve (one block: vectors, then CG scalars, reduction
// partials and a small scalar scratch) and the host mirrors of its scalars.
struct Workspace {
  void *base = nullptr;
  size_t bytes = 0;              // bytes of vectors at base
  CgScalars *sc = nullptr;       // device, nsys entries
  CgScalars *sc_host = nullptr;  // host mirror (pinned for the handle's own workspace)
  double *partials = nullptr;
  int nsys_cap = 0;
  size_t partial_cap = 0;
  double *dscal = nullptr;       // small device scratch (norms), WS_DSCAL doubles
  double *dscal_host = nullptr;  // host mirror
};
constexpr int WS_DSCAL = 256;
// Bytes of one workspace block holding vec_bytes of vectors for nsys systems.
size_t ws_block_bytes(const wd_gauge *g, size_t vec_bytes, int nsys);
// Point w's device buffers into the block at base (ws_block_bytes long).
void ws_carve(const wd_gauge *g, Workspace &w, char *base, size_t vec_bytes, int nsys);
// Bytes of vectors the FP64 even-odd CGLS needs.
size_t cg64_vec_bytes(const wd_gauge *g);
// FP64 even-odd CGLS on a given workspace (w.bytes >= cg64_vec_bytes) on
// stream st (one CG iteration pair as a hipGraph if prm.use_graph);
// synchronises st.
wd_status solve_cg64_on(wd_gauge *g, Workspace &w, const void *b, void *x, double kappa, double tol,
                        const wd_solve_params &prm, wd_solve_info &info, hipStream_t st);
// The argument checks of wd_solve (abi.cpp); fills prm, sets the device.
wd_status solve_args(const wd_gauge *U, const void *b, void *x, double kappa, double tol, const wd_solve_params *p,
                     wd_solve_params &prm);
// r = b - D_W x in FP64 (nsys systems sys_stride bytes apart), |r|^2 -> sc[y].rnorm2
wd_status true_residual64(const wd_gauge *g, const void *b, const void *x, void *r, int nsys, size_t sys_stride,
                          double kappa, CgScalars *sc, RedBuf red, hipStream_t st);
// FP64 even-odd CGLS on stream st (synchronises st)
// FP64 CGLS on the full-lattice D_W (no even-odd reduction)
wd_status solve_cgls_full64(wd_gauge *g, const void *b, void *x, double kappa, double tol,
                            const wd_solve_params &prm, wd_solve_info &info, hipStream_t st);
wd_status solve_cg64(wd_gauge *g, const void *b, void *x, double kappa, double tol, const wd_solve_params &prm,
                     wd_solve_info &info, hipStream_t st);

}  // namespace wd

namespace wd {
// release the PTC preconditioner state a handle may hold (ptc.hip)
void ptc_release(wd_gauge *g);
}  // namespace wd
