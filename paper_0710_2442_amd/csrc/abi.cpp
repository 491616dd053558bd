// C-ABI entry points: argument validation, handle lifetime, error strings.
// Every function returns a wd_status; nothing throws across the boundary.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <vector>

#include "wd_blas.h"
#include "wd_internal.h"
#include "wd_solver.h"

namespace wd {

static thread_local char g_err[512] = "";

wd_status set_error(wd_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

wd_status hip_check(hipError_t e, const char *what) {
  if (e == hipSuccess) return WD_OK;
  if (e == hipErrorOutOfMemory) return set_error(WD_ERR_OOM, "%s: %s", what, hipGetErrorString(e));
  return set_error(WD_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

static wd_status check_dims(const int dims[4]) {
  if (!dims) return set_error(WD_ERR_ARG, "dims is NULL");
  size_t V = 1;
  for (int k = 0; k < 4; ++k) {
    if (dims[k] < 2 || (dims[k] & 1))
      return set_error(WD_ERR_DIMS, "dims[%d] = %d: every extent must be even and >= 2", k, dims[k]);
    V *= (size_t)dims[k];
  }
  if (V / 2 > (size_t)(1u << 30)) return set_error(WD_ERR_DIMS, "lattice too large (%zu sites)", V);
  return WD_OK;
}

static bool prec_ok(int p) { return p >= WD_F64 && p <= WD_BF16; }

static wd_status check_handle(const wd_gauge *g) {
  if (!g) return set_error(WD_ERR_ARG, "gauge handle is NULL");
  return WD_OK;
}

static wd_status set_device(const wd_gauge *g) { return hip_check(hipSetDevice(g->device), "hipSetDevice"); }


wd_status solve_args(const wd_gauge *U, const void *b, void *x, double kappa, double tol,
                     const wd_solve_params *p, wd_solve_params &prm) {
  WD_TRY(check_handle(U));
  if (!b || !x) return set_error(WD_ERR_ARG, "solve: NULL field pointer");
  if (b == x) return set_error(WD_ERR_ARG, "solve: b and x must not overlap");
  if (!isfinite(kappa) || !isfinite(tol)) return set_error(WD_ERR_NONFINITE, "solve: kappa or tol not finite");
  if (!(tol > 0.0)) return set_error(WD_ERR_ARG, "solve: tol must be > 0");
  wd_solve_params_default(&prm);
  if (p) {
    if (p->struct_size < sizeof(size_t) || p->struct_size > sizeof(wd_solve_params))
      return set_error(WD_ERR_ARG, "solve: params.struct_size = %zu", p->struct_size);
    memcpy(&prm, p, p->struct_size);
    prm.struct_size = sizeof(prm);
  }
  if (prm.solver < WD_SOLVER_CG || prm.solver > WD_SOLVER_CGLS_FULL)
    return set_error(WD_ERR_ARG, "solve: solver = %d", prm.solver);
  if (prm.inner_prec == WD_F64 && prm.solver == WD_SOLVER_DEFECT_CG)
    return set_error(WD_ERR_PREC, "solve: defect correction needs a reduced inner precision");
  if (!prec_ok(prm.inner_prec)) return set_error(WD_ERR_PREC, "solve: inner_prec = %d", (int)prm.inner_prec);
  if (!(prm.inner_tol > 0.0 && prm.inner_tol < 1.0)) return set_error(WD_ERR_ARG, "solve: inner_tol must be in (0,1)");
  if (prm.max_iter < 1) return set_error(WD_ERR_ARG, "solve: max_iter must be >= 1");
  if (prm.check_every < 1) prm.check_every = 1;
  if (prm.fgcr_m < 1 || prm.fgcr_m > 64) return set_error(WD_ERR_ARG, "solve: fgcr_m = %d", prm.fgcr_m);
  if (prm.solver == WD_SOLVER_DEFECT_FGCR && prm.fgcr_m > 16)
    return set_error(WD_ERR_ARG, "solve: the mixed FGCR keeps at most 16 directions (fgcr_m = %d)", prm.fgcr_m);
  if (prm.solver == WD_SOLVER_DEFECT_FGCR && prm.inner_prec != WD_F32 && prm.inner_prec != WD_BF16)
    return set_error(WD_ERR_PREC, "solve: the mixed FGCR stores its inner vectors in FP32 or BF16");
  return set_device(U);
}

}  // namespace wd

using namespace wd;

extern "C" {

const char *wd_last_error(void) { return g_err; }

const char *wd_status_string(int s) {
  switch (s) {
    case WD_OK: return "ok";
    case WD_NOT_CONVERGED: return "not converged";
    case WD_ERR_ARG: return "invalid argument";
    case WD_ERR_DIMS: return "invalid lattice dimensions";
    case WD_ERR_PREC: return "unsupported precision";
    case WD_ERR_NONFINITE: return "non-finite value";
    case WD_ERR_OOM: return "out of device memory";
    case WD_ERR_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

size_t wd_vh_pad(const int dims[4]) {
  if (check_dims(dims) != WD_OK) return 0;
  return (size_t)make_geom(dims, -1).vpad;
}

size_t wd_field_bytes(const int dims[4], wd_prec prec, int nrhs, int parity) {
  if (check_dims(dims) != WD_OK || !prec_ok(prec) || nrhs < 1 || parity < 0 || parity > 2) return 0;
  const Geom g = make_geom(dims, -1);
  return half_bytes(g, prec) * (parity == WD_FULL ? 2 : 1) * (size_t)nrhs;
}

wd_status wd_gauge_create(const double *U_host, const int dims[4], int t_bc, wd_prec prec, void *hip_stream,
                          wd_gauge **out) {
  if (!out) return set_error(WD_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!U_host) return set_error(WD_ERR_ARG, "U_host is NULL");
  WD_TRY(check_dims(dims));
  if (t_bc != 1 && t_bc != -1) return set_error(WD_ERR_ARG, "t_bc = %d: must be +1 or -1", t_bc);
  if (!prec_ok(prec)) return set_error(WD_ERR_PREC, "prec = %d", (int)prec);
  wd_gauge *g = new (std::nothrow) wd_gauge();
  if (!g) return set_error(WD_ERR_OOM, "host allocation failed");
  g->geom = make_geom(dims, t_bc);
  for (int k = 0; k < 4; ++k) g->dims[k] = dims[k];
  g->tbc = t_bc;
  g->prec = prec;
  g->stream = (hipStream_t)hip_stream;
  for (int p = 0; p < 4; ++p) {
    // default hop variant: 256 threads, eight XCD regions when the lattice allows
    g->hop_block[p] = 256;
    g->hop_groups[p] = dslash_variant_ok(g->geom, 256, 8) ? 8 : 0;
    g->hop_occ[p] = 0;
    g->hop_ntst[p] = 1;
    g->hop_lds[p] = 0;
    g->hop_pre[p] = 0;
    g->hop_spl[p] = 1;
    g->hop_stage[p] = 0;
    g->mrhs_block[p] = (p == WD_F64) ? 16 : 128;
    g->mrhs_rpl[p] = 4;
    g->mrhs_groups[p] = dslash_variant_ok(g->geom, g->mrhs_block[p], 4) ? 4 : 0;
  }
  wd_status rc = WD_OK;
  void *canon = nullptr;
  const size_t V = (size_t)dims[0] * dims[1] * dims[2] * dims[3];
  const size_t ubytes = V * 4 * 18 * sizeof(double);
  do {
    if ((rc = hip_check(hipGetDevice(&g->device), "hipGetDevice")) != WD_OK) break;
    if ((rc = hip_check(hipDeviceGetAttribute(&g->lds_per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, g->device),
                        "hipDeviceGetAttribute")) != WD_OK)
      break;
    if ((rc = hip_check(hipDeviceGetAttribute(&g->n_cu, hipDeviceAttributeMultiprocessorCount, g->device),
                        "hipDeviceGetAttribute")) != WD_OK)
      break;
    if ((rc = hip_check(hipStreamCreateWithFlags(&g->own_stream, hipStreamNonBlocking), "stream")) != WD_OK) break;
    if ((rc = hip_check(hipMalloc(&g->links64, link_bytes(g->geom, true)), "links64")) != WD_OK) break;
    if ((rc = hip_check(hipMalloc(&g->links32, link_bytes(g->geom, false)), "links32")) != WD_OK) break;
    if ((rc = hip_check(hipMalloc(&g->scratch_red, sizeof(double) * (4 * BLAS_MAX_BLOCKS + 64)), "scratch")) != WD_OK)
      break;
    if ((rc = hip_check(hipMalloc(&canon, ubytes), "gauge staging")) != WD_OK) break;
    if ((rc = hip_check(hipMemcpyAsync(canon, U_host, ubytes, hipMemcpyHostToDevice, g->own_stream), "upload")) !=
        WD_OK)
      break;
    if ((rc = dirac_init(g)) != WD_OK) break;
    if ((rc = launch_pack_gauge(g, canon, g->own_stream)) != WD_OK) break;
    rc = hip_check(hipStreamSynchronize(g->own_stream), "pack gauge");
  } while (0);
  if (canon) (void)hipFree(canon);
  if (rc != WD_OK) {
    char msg[512];
    snprintf(msg, sizeof msg, "%s", g_err);
    wd_gauge_destroy(g);
    return set_error(rc, "%s", msg);
  }
  *out = g;
  return WD_OK;
}

wd_status wd_gauge_destroy(wd_gauge *g) {
  if (!g) return WD_OK;
  (void)hipSetDevice(g->device);
  if (g->own_stream) (void)hipStreamSynchronize(g->own_stream);
  workspace_free(g);
  fgcr_free(g);
  ptc_release(g);
  if (g->links64) (void)hipFree(g->links64);
  if (g->links32) (void)hipFree(g->links32);
  if (g->scratch_red) (void)hipFree(g->scratch_red);
  if (g->own_stream) (void)hipStreamDestroy(g->own_stream);
  delete g;
  return WD_OK;
}

wd_status wd_gauge_set_stream(wd_gauge *g, void *hip_stream) {
  WD_TRY(check_handle(g));
  g->stream = (hipStream_t)hip_stream;
  return WD_OK;
}

wd_status wd_spinor_pack(const wd_gauge *g, const void *canon, void *field, int parity, wd_prec prec) {
  WD_TRY(check_handle(g));
  if (!canon || !field) return set_error(WD_ERR_ARG, "pack: NULL pointer");
  if (parity < 0 || parity > 2) return set_error(WD_ERR_ARG, "pack: parity = %d", parity);
  if (!prec_ok(prec)) return set_error(WD_ERR_PREC, "pack: prec = %d", (int)prec);
  WD_TRY(set_device(g));
  return launch_pack_spinor(g, canon, field, parity, prec, g->stream);
}

wd_status wd_spinor_unpack(const wd_gauge *g, const void *field, void *canon, int parity, wd_prec prec) {
  WD_TRY(check_handle(g));
  if (!canon || !field) return set_error(WD_ERR_ARG, "unpack: NULL pointer");
  if (parity < 0 || parity > 2) return set_error(WD_ERR_ARG, "unpack: parity = %d", parity);
  if (!prec_ok(prec)) return set_error(WD_ERR_PREC, "unpack: prec = %d", (int)prec);
  WD_TRY(set_device(g));
  return launch_unpack_spinor(g, field, canon, parity, prec, g->stream);
}

wd_status wd_gaussian_field(const wd_gauge *g, void *field, int parity, wd_prec prec, unsigned long long seed,
                            unsigned long long stream) {
  WD_TRY(check_handle(g));
  if (!field) return set_error(WD_ERR_ARG, "gaussian field: NULL pointer");
  if (parity < 0 || parity > 2) return set_error(WD_ERR_ARG, "gaussian field: parity = %d", parity);
  if (prec != WD_F64 && prec != WD_F32) return set_error(WD_ERR_PREC, "gaussian field: prec = %d", (int)prec);
  WD_TRY(set_device(g));
  return launch_gaussian(g, field, parity, prec, seed, stream, g->stream);
}

size_t wd_halo_face_bytes(const int dims[4], wd_prec prec) {
  if (check_dims(dims) != WD_OK || (prec != WD_F64 && prec != WD_F32)) return 0;
  const Geom G = make_geom(dims, -1);
  return halo_face_bytes(G, prec);
}

static wd_status slab_check(const wd_gauge *g, int t0, int nt, wd_prec prec) {
  WD_TRY(check_handle(g));
  if (prec != WD_F64 && prec != WD_F32) return set_error(WD_ERR_PREC, "slab: FP64 or FP32 only");
  if (t0 < 0 || nt < 1 || t0 + nt > g->geom.L[3])
    return set_error(WD_ERR_ARG, "slab: slices [%d, %d) outside 0..%d", t0, t0 + nt, g->geom.L[3]);
  if (g->geom.s4 % 64)
    return set_error(WD_ERR_DIMS, "slab: L1 L2 L3 / 2 = %d sites per slice must be a multiple of 64", g->geom.s4);
  return set_device(g);
}

wd_status wd_halo_pack(const wd_gauge *g, const void *in_slab, int nt, int face, int dagger, wd_prec prec,
                       void *face_buf) {
  WD_TRY(slab_check(g, 0, nt, prec));
  if (!in_slab || !face_buf) return set_error(WD_ERR_ARG, "halo pack: NULL pointer");
  if (face != 0 && face != 1) return set_error(WD_ERR_ARG, "halo pack: face = %d", face);
  return launch_halo_pack(g, in_slab, nt, face, dagger, prec, face_buf, g->stream);
}

wd_status wd_dslash_slab(const wd_gauge *g, const void *in_slab, const void *face_lo, const void *face_hi,
                         void *out_slab, double a, int parity, int t0, int nt, int dagger, wd_prec prec) {
  WD_TRY(slab_check(g, t0, nt, prec));
  if (!in_slab || !face_lo || !face_hi || !out_slab) return set_error(WD_ERR_ARG, "slab hop: NULL pointer");
  if (in_slab == out_slab) return set_error(WD_ERR_ARG, "slab hop: in and out must differ");
  if (parity != 0 && parity != 1) return set_error(WD_ERR_ARG, "slab hop: parity = %d", parity);
  if (!isfinite(a)) return set_error(WD_ERR_NONFINITE, "slab hop: a is not finite");
  return launch_dslash_slab(g, in_slab, face_lo, face_hi, out_slab, a, parity, t0, nt, dagger, prec, g->stream);
}

static wd_status dslash_common(const wd_gauge *U, const void *in, void *out, double kappa, int parity, wd_prec prec,
                               int flags) {
  WD_TRY(check_handle(U));
  if (!in || !out) return set_error(WD_ERR_ARG, "dslash: NULL field pointer");
  if (in == out) return set_error(WD_ERR_ARG, "dslash: psi_in and psi_out must not overlap");
  if (parity < 0 || parity > 2) return set_error(WD_ERR_ARG, "dslash: parity = %d", parity);
  if (!prec_ok(prec)) return set_error(WD_ERR_PREC, "dslash: prec = %d", (int)prec);
  if (!isfinite(kappa)) return set_error(WD_ERR_NONFINITE, "dslash: kappa is not finite");
  if (flags & ~(WD_DAGGER | WD_ONE_PASS)) return set_error(WD_ERR_ARG, "dslash: unknown flags 0x%x", flags);
  WD_TRY(set_device(U));
  const int dag = (flags & WD_DAGGER) ? 1 : 0;
  if (parity != WD_FULL) {
    DslashArgs a;
    a.in = in; a.out = out; a.a = kappa; a.parity = parity; a.dagger = dag;
    return launch_dslash(U, prec, a, U->stream);
  }
  // D_W in = in - kappa H in, both halves
  const size_t hb = half_bytes(U->geom, prec);
  const size_t ob = (const char *)out > (const char *)in ? (size_t)((const char *)out - (const char *)in)
                                                          : (size_t)((const char *)in - (const char *)out);
  if (ob < 2 * hb) return set_error(WD_ERR_ARG, "dslash: full fields overlap");
  if (flags & WD_ONE_PASS) {
    DiracArgs a;
    a.in = in; a.out = out; a.X = in; a.a = -kappa; a.dagger = dag;
    return launch_dirac(U, prec, a, U->stream);
  }
  for (int p = 0; p < 2; ++p) {
    DslashArgs a;
    a.in = (const char *)in + (1 - p) * hb;
    a.out = (char *)out + p * hb;
    a.X = (const char *)in + p * hb;
    a.a = -kappa;
    a.parity = p;
    a.dagger = dag;
    WD_TRY(launch_dslash(U, prec, a, U->stream));
  }
  return WD_OK;
}

wd_status wd_dslash(const wd_gauge *U, const void *psi_in, void *psi_out, double kappa, const int dims[4],
                    int parity) {
  WD_TRY(check_handle(U));
  WD_TRY(check_dims(dims));
  for (int k = 0; k < 4; ++k)
    if (dims[k] != U->dims[k]) return set_error(WD_ERR_DIMS, "dslash: dims differ from the handle's dims");
  return dslash_common(U, psi_in, psi_out, kappa, parity, U->prec, 0);
}

wd_status wd_dslash_ex(const wd_gauge *U, const void *psi_in, void *psi_out, double kappa, int parity, wd_prec prec,
                       int flags) {
  return dslash_common(U, psi_in, psi_out, kappa, parity, prec, flags);
}

wd_status wd_dslash_mrhs(const wd_gauge *U, const void *in, void *out, double kappa, int parity, wd_prec prec,
                         int nrhs) {
  WD_TRY(check_handle(U));
  if (!in || !out) return set_error(WD_ERR_ARG, "dslash_mrhs: NULL field pointer");
  if (in == out) return set_error(WD_ERR_ARG, "dslash_mrhs: in and out must not overlap");
  if (parity != WD_EVEN && parity != WD_ODD) return set_error(WD_ERR_ARG, "dslash_mrhs: parity = %d", parity);
  if (!prec_ok(prec)) return set_error(WD_ERR_PREC, "dslash_mrhs: prec = %d", (int)prec);
  if (nrhs < 1 || nrhs > 64) return set_error(WD_ERR_ARG, "dslash_mrhs: nrhs = %d", nrhs);
  if (!isfinite(kappa)) return set_error(WD_ERR_NONFINITE, "dslash_mrhs: kappa is not finite");
  WD_TRY(set_device(U));
  return launch_dslash_mrhs(U, prec, in, out, kappa, parity, 0, nrhs, U->stream);
}

// ---------------------------------------------------------------- BLAS
static wd_status blas_args(const wd_gauge *g, const void *x, int nhalf, wd_prec prec) {
  WD_TRY(check_handle(g));
  if (!x) return set_error(WD_ERR_ARG, "blas: NULL field pointer");
  if (nhalf < 1) return set_error(WD_ERR_ARG, "blas: nhalf = %d", nhalf);
  if (!prec_ok(prec)) return set_error(WD_ERR_PREC, "blas: prec = %d", (int)prec);
  return set_device(g);
}

wd_status wd_caxpy(const wd_gauge *g, double c_re, double c_im, const void *x, void *y, int nhalf, wd_prec prec) {
  WD_TRY(blas_args(g, x, nhalf, prec));
  if (!y) return set_error(WD_ERR_ARG, "caxpy: y is NULL");
  if (!isfinite(c_re) || !isfinite(c_im)) return set_error(WD_ERR_NONFINITE, "caxpy: c is not finite");
  return blas_caxpy(g->geom, prec, c_re, c_im, vref(x, nhalf), vref(y, nhalf), 1, g->stream);
}

wd_status wd_cdot(const wd_gauge *g, const void *x, const void *y, int nhalf, wd_prec prec, double out[2]) {
  WD_TRY(blas_args(g, x, nhalf, prec));
  if (!y || !out) return set_error(WD_ERR_ARG, "cdot: NULL pointer");
  RedBuf red{g->scratch_red + 64};
  WD_TRY(blas_cdot(g->geom, prec, vref(x, nhalf), vref(y, nhalf), 1, red, g->scratch_red, g->stream));
  WD_HIP(hipMemcpyAsync(out, g->scratch_red, 2 * sizeof(double), hipMemcpyDeviceToHost, g->stream));
  WD_HIP(hipStreamSynchronize(g->stream));
  return WD_OK;
}

wd_status wd_norm2(const wd_gauge *g, const void *x, int nhalf, wd_prec prec, double *out) {
  WD_TRY(blas_args(g, x, nhalf, prec));
  if (!out) return set_error(WD_ERR_ARG, "norm2: out is NULL");
  RedBuf red{g->scratch_red + 64};
  WD_TRY(blas_norm2(g->geom, prec, vref(x, nhalf), 1, red, g->scratch_red, g->stream));
  WD_HIP(hipMemcpyAsync(out, g->scratch_red, sizeof(double), hipMemcpyDeviceToHost, g->stream));
  WD_HIP(hipStreamSynchronize(g->stream));
  return WD_OK;
}

wd_status wd_convert(const wd_gauge *g, const void *in, wd_prec pin, void *out, wd_prec pout, int nhalf,
                     double scale) {
  WD_TRY(blas_args(g, in, nhalf, pin));
  if (!out) return set_error(WD_ERR_ARG, "convert: out is NULL");
  if (!prec_ok(pout)) return set_error(WD_ERR_PREC, "convert: prec = %d", (int)pout);
  if (!isfinite(scale)) return set_error(WD_ERR_NONFINITE, "convert: scale is not finite");
  if (in == out && pin != pout) return set_error(WD_ERR_ARG, "convert: in place needs equal precisions");
  return blas_convert(g->geom, pin, vref(in, nhalf), pout, vref(out, nhalf), scale, nullptr, 1, g->stream);
}

// ---------------------------------------------------------------- solve
void wd_solve_params_default(wd_solve_params *p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(*p);
  p->solver = WD_SOLVER_CG;
  p->inner_prec = WD_F32;
  p->inner_tol = 1e-3;
  p->max_iter = 100000;
  p->check_every = 16;
  p->use_graph = 1;
  p->fgcr_m = 12;
  p->precond = nullptr;
}

wd_status wd_solve(const wd_gauge *U, const void *b, void *x, double kappa, double tol, const wd_solve_params *p,
                   wd_solve_info *info) {
  wd_solve_params prm;
  WD_TRY(solve_args(U, b, x, kappa, tol, p, prm));
  wd_solve_info tmp;
  memset(&tmp, 0, sizeof tmp);
  wd_status rc = solve(const_cast<wd_gauge *>(U), b, x, kappa, tol, prm, tmp);
  tmp.status = rc;
  if (info) *info = tmp;
  return rc;
}

wd_status wd_solve_mrhs(const wd_gauge *U, const void *b, void *x, int nrhs, double kappa, double tol,
                        const wd_solve_params *p, wd_solve_info *info) {
  wd_solve_params prm;
  WD_TRY(solve_args(U, b, x, kappa, tol, p, prm));
  if (nrhs < 1 || nrhs > 64) return set_error(WD_ERR_ARG, "solve_mrhs: nrhs = %d", nrhs);
  if (prm.solver != WD_SOLVER_DEFECT_CG) return set_error(WD_ERR_ARG, "solve_mrhs: only defect-correction CG");
  std::vector<wd_solve_info> tmp(nrhs);
  for (auto &t : tmp) memset(&t, 0, sizeof t);
  wd_status rc = solve_mrhs(const_cast<wd_gauge *>(U), b, x, nrhs, kappa, tol, prm, tmp.data());
  if (info)
    for (int y = 0; y < nrhs; ++y) {
      if (rc < 0) tmp[y].status = rc;
      info[y] = tmp[y];
    }
  return rc;
}

wd_status wd_solve_batch(const wd_gauge *const *gs, int n, const void *const *b, void *const *x, const double *kappa,
                         double tol, const wd_solve_params *p, wd_solve_info *infos) {
  if (!gs || !b || !x || !kappa || !infos) return set_error(WD_ERR_ARG, "solve_batch: NULL argument");
  if (n < 1 || n > 4096) return set_error(WD_ERR_ARG, "solve_batch: n = %d", n);
  wd_solve_params prm;
  for (int l = 0; l < n; ++l) {
    WD_TRY(solve_args(gs[l], b[l], x[l], kappa[l], tol, p, prm));
    if (gs[l]->device != gs[0]->device) return set_error(WD_ERR_ARG, "solve_batch: handles on different devices");
  }
  if (prm.solver != WD_SOLVER_DEFECT_CG) return set_error(WD_ERR_ARG, "solve_batch: only defect-correction CG");
  if (prm.batch_tile != 0 && prm.batch_tile != 64 && prm.batch_tile != 128 && prm.batch_tile != 256)
    return set_error(WD_ERR_ARG, "solve_batch: batch_tile = %d (0, 64, 128 or 256)", prm.batch_tile);
  if (prm.batch_blocks_per_cu < -1 || prm.batch_blocks_per_cu > 64)
    return set_error(WD_ERR_ARG, "solve_batch: batch_blocks_per_cu = %d (-1 .. 64)", prm.batch_blocks_per_cu);
  wd_status rc = solve_batch(gs, n, b, x, kappa, tol, prm, infos);
  if (rc < 0)
    for (int l = 0; l < n; ++l) infos[l].status = rc;
  return rc;
}

}  // extern "C"
