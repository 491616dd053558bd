// Allocation-free FP64 solve: wd_solve's even-odd CGLS with the solver's
// workspace in a static device array instead of device memory the library
// allocates.  For callers that must not allocate on the call.
//
// Every GPU that runs this library holds one copy of `scratch`
// (WD_NOALLOC_SCRATCH_BYTES) until the process ends.  In host code the name
// `scratch` is only a host-side stand-in: its device address on each GPU is
// looked up once with hipGetSymbolAddress (that GPU current) and kept; only
// that address is handed to kernels.  All calls on one GPU share the array:
// calls that overlap on one GPU (two host threads, or two streams) race.  The
// solve writes every part of the workspace before reading it (x is zeroed,
// the CG scalars are uploaded from the host, reductions store their partials
// before the finishing sums read them), so what an earlier call left there
// never matters and nothing needs clearing.
#include <string.h>

#include <chrono>
#include <mutex>

#include "wd_blas.h"
#include "wd_solver.h"

namespace wd {

static __device__ __align__(256) unsigned char scratch[WD_NOALLOC_SCRATCH_BYTES];

static constexpr int kMaxDevices = 64;
static std::mutex scratch_lock;
static char *scratch_addr[kMaxDevices];  // device address of `scratch` per GPU (null until looked up)

// Device address of this GPU's copy of `scratch`; device `dev` must be current.
static wd_status scratch_of(int dev, char *&out) {
  if (dev < 0 || dev >= kMaxDevices) return set_error(WD_ERR_ARG, "allocation-free solve: device %d", dev);
  std::lock_guard<std::mutex> hold(scratch_lock);
  if (!scratch_addr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_check(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
    scratch_addr[dev] = (char *)p;
  }
  out = scratch_addr[dev];
  return WD_OK;
}

}  // namespace wd

using namespace wd;

extern "C" {

wd_status wd_solve_noalloc(const wd_gauge *U, const void *b, void *x, double kappa, double tol,
                           const wd_solve_params *p, wd_solve_info *info) {
  wd_solve_params prm;
  WD_TRY(solve_args(U, b, x, kappa, tol, p, prm));  // also makes the handle's device current
  if (prm.solver != WD_SOLVER_CG)
    return set_error(WD_ERR_ARG, "solve_noalloc: only the FP64 CG (WD_SOLVER_CG), solver = %d", prm.solver);
  prm.use_graph = 0;  // iterations are launched one by one: instantiating a graph allocates
  wd_gauge *g = const_cast<wd_gauge *>(U);
  const size_t vec = cg64_vec_bytes(g);
  const size_t need = ws_block_bytes(g, vec, 1);
  if (need > (size_t)WD_NOALLOC_SCRATCH_BYTES)
    return set_error(WD_ERR_ARG, "solve_noalloc: this lattice needs %zu bytes of workspace, the limit is %zu", need,
                     (size_t)WD_NOALLOC_SCRATCH_BYTES);
  char *base = nullptr;
  WD_TRY(scratch_of(g->device, base));
  CgScalars sc_host[1];
  double dscal_host[WS_DSCAL];
  Workspace w;
  ws_carve(g, w, base, vec, 1);
  w.sc_host = sc_host;
  w.dscal_host = dscal_host;
  wd_solve_info tmp;
  memset(&tmp, 0, sizeof tmp);
  const auto t0 = std::chrono::steady_clock::now();
  wd_status rc = solve_cg64_on(g, w, b, x, kappa, tol, prm, tmp, g->stream);
  // also after a failure: nothing queued may outlive the host mirrors above
  const hipError_t e = hipStreamSynchronize(g->stream);
  if (rc >= 0 && e != hipSuccess) rc = hip_check(e, "solve_noalloc sync");
  tmp.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  tmp.status = rc;
  if (info) *info = tmp;
  return rc;
}

}  // extern "C"
