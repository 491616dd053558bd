// Solvers for D_W x = b built on the single-parity hop kernels.
//
// * FP64 full-lattice CGLS: CG on D^dag D x = D^dag b on full fields, each
//   operator application one hop launch per parity (no even-odd reduction).
// * FP64 even-odd CGLS: CG on the normal equations of the Schur operator
//   M = 1 - k^2 H_eo H_oe (M^dag = 1 - k^2 H^dag_eo H^dag_oe), right-hand
//   side b_e + k H_eo b_o, odd sites x_o = b_o + k H_oe x_e.  The paper
//   leaves the solver that applies Eq. 3 over and over unspecified (Sec. 5,
//   data in on-chip memory); CGLS is the reading used here.
// * Defect correction: FP64 outer residual r = b - D x, inner even-odd CGLS
//   in FP32 arithmetic on r/|r| with vectors stored in FP32, FP16 (+ per-site
//   scale) or BF16, x += |r| e in FP64.
// * Multi right-hand side: the same recurrences for nrhs systems with their
//   own scalars, sharing every hop launch (links loaded once per site).
//
// All CG scalars stay on the device; kernels of converged systems return
// immediately, so the host polls convergence only every few iterations.  One
// pair of CG iterations can be captured into a hipGraph and replayed.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "wd_blas.h"
#include "wd_solver.h"

namespace wd {

// ------------------------------------------------------------ workspace
// largest grid.x of any reducing launch: single-RHS hop, level-1, multi-RHS hop
static size_t ws_partials(const wd_gauge *g, int nsys) {
  const size_t nblk = std::max<size_t>(std::max<unsigned>(dslash_grid_blocks(g), BLAS_MAX_BLOCKS),
                                       mrhs_grid_blocks(g));
  return nblk * 2 * (size_t)nsys;
}

size_t ws_block_bytes(const wd_gauge *g, size_t vec_bytes, int nsys) {
  return round_up(vec_bytes, 256) + round_up(sizeof(CgScalars) * nsys, 256) +
         round_up(ws_partials(g, nsys) * sizeof(double), 256) + WS_DSCAL * sizeof(double);
}

void ws_carve(const wd_gauge *g, Workspace &w, char *base, size_t vec_bytes, int nsys) {
  char *c = base;
  w.base = c; c += round_up(vec_bytes, 256);
  w.sc = (CgScalars *)c; c += round_up(sizeof(CgScalars) * nsys, 256);
  w.partials = (double *)c; c += round_up(ws_partials(g, nsys) * sizeof(double), 256);
  w.dscal = (double *)c;
  w.bytes = vec_bytes;
  w.nsys_cap = nsys;
  w.partial_cap = ws_partials(g, nsys);
}

static wd_status ws_reserve(wd_gauge *g, size_t vec_bytes, int nsys) {
  Workspace *&w = g->ws;
  if (!w) w = new Workspace();
  if (w->base && w->bytes >= vec_bytes && w->nsys_cap >= nsys && w->partial_cap >= ws_partials(g, nsys)) return WD_OK;
  if (w->base) {
    WD_HIP(hipFree(w->base));
    w->base = nullptr;
  }
  if (w->sc_host) { WD_HIP(hipHostFree(w->sc_host)); w->sc_host = nullptr; }
  if (w->dscal_host) { WD_HIP(hipHostFree(w->dscal_host)); w->dscal_host = nullptr; }
  const size_t total = ws_block_bytes(g, vec_bytes, nsys);
  void *base = nullptr;
  if (hipMalloc(&base, total) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(WD_ERR_OOM, "solver workspace: cannot allocate %zu bytes", total);
  }
  ws_carve(g, *w, (char *)base, vec_bytes, nsys);
  WD_HIP(hipHostMalloc((void **)&w->sc_host, round_up(sizeof(CgScalars) * nsys, 256), hipHostMallocDefault));
  WD_HIP(hipHostMalloc((void **)&w->dscal_host, WS_DSCAL * sizeof(double), hipHostMallocDefault));
  return WD_OK;
}

void workspace_free(wd_gauge *g) {
  if (!g->ws) return;
  Workspace *w = g->ws;
  if (w->base) (void)hipFree(w->base);
  if (w->sc_host) (void)hipHostFree(w->sc_host);
  if (w->dscal_host) (void)hipHostFree(w->dscal_host);
  delete w;
  g->ws = nullptr;
}

static RedBuf red_of(const Workspace *w) { return RedBuf{w->partials}; }

// ------------------------------------------------------------ operators
// One hop application for nsys systems: single-RHS kernel when nsys == 1.
struct HopCall {
  const void *in;
  void *out;
  const void *X;
  double a;
  int parity;
  int dagger;
  double *norm_out;  // system 0's slot; stride sizeof(CgScalars)
  const int *skip;   // system 0's done flag
};

static wd_status hop(const wd_gauge *g, wd_prec prec, int nsys, const HopCall &c, RedBuf red, hipStream_t st) {
  if (nsys == 1) {
    DslashArgs a;
    a.in = c.in; a.out = c.out; a.X = c.X; a.a = c.a; a.parity = c.parity; a.dagger = c.dagger;
    a.norm_out = c.norm_out; a.skip = c.skip; a.red = red;
    return launch_dslash(g, prec, a, st);
  }
  MrhsArgs m;
  m.in = c.in; m.out = c.out; m.X = c.X; m.a = c.a; m.parity = c.parity; m.dagger = c.dagger;
  m.nrhs = nsys;
  m.norm_out = c.norm_out;
  m.norm_stride = sizeof(CgScalars) / sizeof(double);
  m.skip = c.skip;
  m.skip_stride = sizeof(CgScalars) / sizeof(int);
  m.red = red;
  return launch_dslash_mrhs_ex(g, prec, m, st);
}

struct CglsVecs {
  wd_prec px, pv;
  int nsys;
  void *x;            // parity-0 solution (px); the full solution when full
  void *p, *s, *r, *q;  // parity-0 vectors (pv); full fields when full
  void *t;            // parity-1 temporary (pv); unused when full
  size_t sx, sv;      // per-system strides of x and of the pv vectors
  int full = 0;       // 1: the operator is D_W itself on full fields, not the Schur operator
};

// out = A in (dagger: A^dag in), |out|^2 -> norm: A = M = 1 - k^2 H_eo H_oe on
// even halves (two hops, the first into t), or A = D_W = 1 - k H on full
// fields (the one-launch marching kernel where it fills the device, else one
// hop per parity with the norm summed over both).
static wd_status apply_op(const wd_gauge *g, const CglsVecs &v, double kappa, const void *in, void *out, int dagger,
                          double *norm, const int *skip, RedBuf red, hipStream_t st) {
  if (!v.full) {
    WD_TRY(hop(g, v.pv, v.nsys, HopCall{in, v.t, nullptr, 1.0, 1, dagger, nullptr, skip}, red, st));
    return hop(g, v.pv, v.nsys, HopCall{v.t, out, in, -kappa * kappa, 0, dagger, norm, skip}, red, st);
  }
  if (dirac_fills_device(g, v.pv)) {
    DiracArgs a;
    a.in = in;
    a.out = out;
    a.X = in;
    a.a = -kappa;
    a.dagger = dagger;
    a.norm_out = norm;
    a.skip = skip;
    a.red = red;
    return launch_dirac(g, v.pv, a, st);
  }
  const size_t hb = half_bytes(g->geom, v.pv);
  for (int par = 0; par < 2; ++par) {
    DslashArgs a;
    a.in = (const char *)in + (1 - par) * hb;
    a.out = (char *)out + par * hb;
    a.X = (const char *)in + par * hb;
    a.a = -kappa;
    a.parity = par;
    a.dagger = dagger;
    a.norm_out = norm;
    a.norm_accumulate = par;
    a.skip = skip;
    a.red = red;
    WD_TRY(launch_dslash(g, v.pv, a, st));
  }
  return WD_OK;
}

// q = A p -> qq;  cg_update;  r = A^dag s -> rr[1-j];  p = r + beta p
static wd_status cgls_iteration(const wd_gauge *g, const CglsVecs &v, double kappa, CgScalars *sc, int j,
                                RedBuf red, hipStream_t st) {
  const int *skip = &sc->done;
  const int nh = v.full ? 2 : 1;
  WD_TRY(apply_op(g, v, kappa, v.p, v.q, 0, &sc->qq, skip, red, st));
  WD_TRY(blas_cg_update(g->geom, v.px, vref(v.x, nh, v.sx), v.pv, vref(v.p, nh, v.sv), vref(v.s, nh, v.sv),
                        vref(v.q, nh, v.sv), sc, j, v.nsys, red, st));
  WD_TRY(apply_op(g, v, kappa, v.s, v.r, 1, &sc->rr[1 - j], skip, red, st));
  WD_TRY(blas_cg_pupdate(g->geom, v.pv, vref(v.r, nh, v.sv), vref(v.p, nh, v.sv), sc, j, v.nsys, st));
  return WD_OK;
}

// Runs CGLS on M x = s (s holds the right-hand side on entry; x is zeroed).
// sc_init[sys] carries stop2 / max_iters; returns per-system results in
// w->sc_host.  dslash_calls is incremented by the hop count issued.
static wd_status cgls_run(const wd_gauge *g, Workspace *w, const CglsVecs &v, double kappa,
                          const CgScalars *sc_init, const wd_solve_params &prm, hipStream_t st, int &dslash_calls) {
  RedBuf red = red_of(w);
  CgScalars *sc = w->sc;
  for (int y = 0; y < v.nsys; ++y) w->sc_host[y] = sc_init[y];
  WD_HIP(hipMemcpyAsync(sc, w->sc_host, sizeof(CgScalars) * v.nsys, hipMemcpyHostToDevice, st));
  const int nh = v.full ? 2 : 1;
  // x = 0
  WD_TRY(blas_convert(g->geom, v.pv, vref(v.s, nh, v.sv), v.px, vref(v.x, nh, v.sx), 0.0, nullptr, v.nsys, st));
  // r = A^dag s, rr[0] = |r|^2;  p = r
  WD_TRY(apply_op(g, v, kappa, v.s, v.r, 1, &sc->rr[0], nullptr, red, st));
  WD_TRY(blas_convert(g->geom, v.pv, vref(v.r, nh, v.sv), v.pv, vref(v.p, nh, v.sv), 1.0, nullptr, v.nsys, st));
  dslash_calls += 2;

  int max_iter = 0;
  for (int y = 0; y < v.nsys; ++y) max_iter = std::max(max_iter, sc_init[y].max_iters);
  const int check = std::max(2, prm.check_every & ~1);
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (prm.use_graph) {
    WD_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    wd_status s0 = cgls_iteration(g, v, kappa, sc, 0, red, st);
    wd_status s1 = (s0 == WD_OK) ? cgls_iteration(g, v, kappa, sc, 1, red, st) : s0;
    hipError_t e = hipStreamEndCapture(st, &graph);
    if (s1 != WD_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s1;
    }
    WD_HIP(e);
    WD_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  }
  wd_status rc = WD_OK;
  int issued = 0;
  while (issued < max_iter + 2) {
    for (int k = 0; k < check; k += 2) {
      if (exec) {
        if (hipGraphLaunch(exec, st) != hipSuccess) { rc = hip_check(hipGetLastError(), "graph launch"); break; }
      } else {
        rc = cgls_iteration(g, v, kappa, sc, 0, red, st);
        if (rc == WD_OK) rc = cgls_iteration(g, v, kappa, sc, 1, red, st);
        if (rc != WD_OK) break;
      }
      issued += 2;
    }
    if (rc != WD_OK) break;
    if (hipMemcpyAsync(w->sc_host, sc, sizeof(CgScalars) * v.nsys, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      rc = hip_check(hipGetLastError(), "cg poll");
      break;
    }
    bool all = true;
    for (int y = 0; y < v.nsys; ++y) all = all && (w->sc_host[y].done != 0);
    if (all) break;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (rc != WD_OK) return rc;
  WD_HIP(hipMemcpyAsync(w->sc_host, sc, sizeof(CgScalars) * v.nsys, hipMemcpyDeviceToHost, st));
  WD_HIP(hipStreamSynchronize(st));
  int total = 0;
  for (int y = 0; y < v.nsys; ++y) total = std::max(total, w->sc_host[y].iters);
  dslash_calls += 4 * total;
  return WD_OK;
}

// r = b - D x (FP64, full fields) for nsys systems, |r|^2 -> sc[y].rnorm2
wd_status true_residual64(const wd_gauge *g, const void *b, const void *x, void *r, int nsys, size_t sys_stride,
                          double kappa, CgScalars *sc, RedBuf red, hipStream_t st) {
  const size_t hb = half_bytes(g->geom, WD_F64);
  if (nsys == 1) {
    // r = b - x + kappa H x with |r|^2: the one-launch marching D_W where its
    // work items fill the device (each link and spinor fetched once), else
    // two single-parity launches with the xpay and norm epilogues
    if (dirac_fills_device(g, WD_F64)) {
      DiracArgs a;
      a.in = x;
      a.out = r;
      a.X = b;
      a.Y = x;
      a.a = kappa;
      a.norm_out = &sc->rnorm2;
      a.red = red;
      return launch_dirac(g, WD_F64, a, st);
    }
    for (int par = 0; par < 2; ++par) {
      DslashArgs a;
      a.in = (const char *)x + (1 - par) * hb;
      a.out = (char *)r + par * hb;
      a.X = (const char *)b + par * hb;
      a.Y = (const char *)x + par * hb;
      a.a = kappa;
      a.parity = par;
      a.norm_out = &sc->rnorm2;
      a.norm_accumulate = par;
      a.red = red;
      WD_TRY(launch_dslash(g, WD_F64, a, st));
    }
    return WD_OK;
  }
  for (int par = 0; par < 2; ++par) {
    MrhsArgs m;
    m.in = (const char *)x + (1 - par) * hb;
    m.out = (char *)r + par * hb;
    m.X = (const char *)b + par * hb;
    m.Y = (const char *)x + par * hb;
    m.a = kappa;
    m.parity = par;
    m.nrhs = nsys;
    m.rhs_stride = sys_stride;
    m.norm_out = &sc->rnorm2;
    m.norm_stride = sizeof(CgScalars) / sizeof(double);
    m.norm_accumulate = par;
    m.red = red;
    WD_TRY(launch_dslash_mrhs_ex(g, WD_F64, m, st));
  }
  return WD_OK;
}

// ------------------------------------------------------------ FP64 eo-CGLS
size_t cg64_vec_bytes(const wd_gauge *g) {
  // vectors: p s r q (even) t (odd) + residual (full): 7 halves, one spare
  return half_bytes(g->geom, WD_F64) * 8;
}

wd_status solve_cg64(wd_gauge *g, const void *b, void *x, double kappa, double tol,
                     const wd_solve_params &prm, wd_solve_info &info, hipStream_t st) {
  WD_TRY(ws_reserve(g, cg64_vec_bytes(g), 1));
  return solve_cg64_on(g, *g->ws, b, x, kappa, tol, prm, info, st);
}

wd_status solve_cg64_on(wd_gauge *g, Workspace &ws, const void *b, void *x, double kappa, double tol,
                        const wd_solve_params &prm, wd_solve_info &info, hipStream_t st) {
  const Geom &G = g->geom;
  const size_t hb = half_bytes(G, WD_F64);
  Workspace *w = &ws;
  RedBuf red = red_of(w);
  char *v0 = (char *)w->base;
  CglsVecs V;
  V.px = V.pv = WD_F64;
  V.nsys = 1;
  V.x = x;  // even half of the caller's x
  V.p = v0 + 0 * hb; V.s = v0 + 1 * hb; V.r = v0 + 2 * hb; V.q = v0 + 3 * hb; V.t = v0 + 4 * hb;
  V.sx = V.sv = 0;
  void *res = v0 + 5 * hb;  // full field (2 halves)

  // |b|^2
  WD_TRY(blas_norm2(G, WD_F64, vref(b, 2), 1, red, w->dscal, st));
  WD_HIP(hipMemcpyAsync(w->dscal_host, w->dscal, sizeof(double), hipMemcpyDeviceToHost, st));
  WD_HIP(hipStreamSynchronize(st));
  const double bb = w->dscal_host[0];
  if (!(bb < 1e300)) return set_error(WD_ERR_NONFINITE, "wd_solve: |b|^2 is not finite");
  if (bb == 0.0) {
    WD_TRY(blas_convert(G, WD_F64, vref(b, 2), WD_F64, vref(x, 2), 0.0, nullptr, 1, st));
    WD_HIP(hipStreamSynchronize(st));
    info.true_rel_resid = 0.0;
    return WD_OK;
  }
  // s = bh = b_e + k H_eo b_o
  {
    DslashArgs a;
    a.in = (const char *)b + hb; a.out = V.s; a.X = b; a.a = kappa; a.parity = 0;
    WD_TRY(launch_dslash(g, WD_F64, a, st));
    info.dslash_calls += 1;
  }
  CgScalars init{};
  init.stop2 = tol * tol * bb;
  init.max_iters = prm.max_iter;
  init.bb = bb;
  WD_TRY(cgls_run(g, w, V, kappa, &init, prm, st, info.dslash_calls));
  info.iters = w->sc_host[0].iters;
  const int done = w->sc_host[0].done;
  // x_o = b_o + k H_oe x_e
  {
    DslashArgs a;
    a.in = x; a.out = (char *)x + hb; a.X = (const char *)b + hb; a.a = kappa; a.parity = 1;
    WD_TRY(launch_dslash(g, WD_F64, a, st));
    info.dslash_calls += 1;
  }
  WD_TRY(true_residual64(g, b, x, res, 1, 0, kappa, w->sc, red, st));
  info.dslash_calls += 2;
  WD_HIP(hipMemcpyAsync(w->sc_host, w->sc, sizeof(CgScalars), hipMemcpyDeviceToHost, st));
  WD_HIP(hipStreamSynchronize(st));
  info.true_rel_resid = sqrt(w->sc_host[0].rnorm2 / bb);
  info.outer_iters = 1;
  if (done == 2) return set_error(WD_NOT_CONVERGED, "CG breakdown after %d iterations", info.iters);
  return info.true_rel_resid <= tol ? WD_OK : WD_NOT_CONVERGED;
}

// ------------------------------------------------------------ FP64 full CGLS
// CG on the normal equations of D_W itself, D^dag D x = D^dag b, on full
// fields: no even-odd reduction (the plain method the even-odd solver is
// measured against).  Vectors: p s r q (full) + the true residual (full).
wd_status solve_cgls_full64(wd_gauge *g, const void *b, void *x, double kappa, double tol,
                            const wd_solve_params &prm, wd_solve_info &info, hipStream_t st) {
  const Geom &G = g->geom;
  const size_t fb = 2 * half_bytes(G, WD_F64);
  WD_TRY(ws_reserve(g, 5 * fb, 1));
  Workspace *w = g->ws;
  RedBuf red = red_of(w);
  char *v0 = (char *)w->base;
  CglsVecs V;
  V.px = V.pv = WD_F64;
  V.nsys = 1;
  V.full = 1;
  V.x = x;
  V.p = v0; V.s = v0 + fb; V.r = v0 + 2 * fb; V.q = v0 + 3 * fb; V.t = nullptr;
  V.sx = V.sv = 0;
  void *res = v0 + 4 * fb;
  WD_TRY(blas_norm2(G, WD_F64, vref(b, 2), 1, red, w->dscal, st));
  WD_HIP(hipMemcpyAsync(w->dscal_host, w->dscal, sizeof(double), hipMemcpyDeviceToHost, st));
  WD_HIP(hipStreamSynchronize(st));
  const double bb = w->dscal_host[0];
  if (!(bb < 1e300)) return set_error(WD_ERR_NONFINITE, "wd_solve: |b|^2 is not finite");
  if (bb == 0.0) {
    WD_TRY(blas_convert(G, WD_F64, vref(b, 2), WD_F64, vref(x, 2), 0.0, nullptr, 1, st));
    WD_HIP(hipStreamSynchronize(st));
    info.true_rel_resid = 0.0;
    return WD_OK;
  }
  // s = b (the residual of x = 0)
  WD_TRY(blas_convert(G, WD_F64, vref(b, 2), WD_F64, vref(V.s, 2), 1.0, nullptr, 1, st));
  CgScalars init{};
  init.stop2 = tol * tol * bb;
  init.max_iters = prm.max_iter;
  init.bb = bb;
  int calls = 0;
  WD_TRY(cgls_run(g, w, V, kappa, &init, prm, st, calls));
  info.dslash_calls += calls;  // hop launches (one per parity per operator application)
  info.iters = w->sc_host[0].iters;
  const int done = w->sc_host[0].done;
  WD_TRY(true_residual64(g, b, x, res, 1, 0, kappa, w->sc, red, st));
  info.dslash_calls += 2;
  WD_HIP(hipMemcpyAsync(w->sc_host, w->sc, sizeof(CgScalars), hipMemcpyDeviceToHost, st));
  WD_HIP(hipStreamSynchronize(st));
  info.true_rel_resid = sqrt(w->sc_host[0].rnorm2 / bb);
  info.outer_iters = 1;
  if (done == 2) return set_error(WD_NOT_CONVERGED, "CG breakdown after %d iterations", info.iters);
  return info.true_rel_resid <= tol ? WD_OK : WD_NOT_CONVERGED;
}

// ------------------------------------------------------------ defect correction
// nsys systems share the operator; b, x: nsys full FP64 fields (stride sb).
static wd_status solve_defect(wd_gauge *g, const void *b, void *x, int nsys, size_t sb, double kappa, double tol,
                              const wd_solve_params &prm, wd_solve_info *infos, hipStream_t st) {
  const Geom &G = g->geom;
  const wd_prec S = prm.inner_prec;
  const size_t h64 = half_bytes(G, WD_F64), h32 = half_bytes(G, WD_F32), hS = half_bytes(G, S);
  // per system: r64 (2 h64), rh32 (2 h32), e32 (2 h32), p s r q (hS each), t (hS)
  const size_t per = 2 * h64 + 4 * h32 + 5 * hS;
  WD_TRY(ws_reserve(g, per * nsys, nsys));
  Workspace *w = g->ws;
  RedBuf red = red_of(w);
  char *c = (char *)w->base;
  char *r64 = c; c += 2 * h64 * nsys;
  char *rh32 = c; c += 2 * h32 * nsys;
  char *e32 = c; c += 2 * h32 * nsys;
  CglsVecs V;
  V.px = WD_F32;
  V.pv = S;
  V.nsys = nsys;
  V.x = e32;  // even half of e32 per system
  V.sx = 2 * h32;
  V.sv = hS;
  V.p = c; c += hS * nsys;
  V.s = c; c += hS * nsys;
  V.r = c; c += hS * nsys;
  V.q = c; c += hS * nsys;
  V.t = c; c += hS * nsys;

  // |b|^2 per system; x = 0; r = b
  WD_TRY(blas_norm2(G, WD_F64, vref(b, 2, sb), nsys, red, w->dscal, st));
  WD_HIP(hipMemcpyAsync(w->dscal_host, w->dscal, sizeof(double) * nsys, hipMemcpyDeviceToHost, st));
  WD_HIP(hipStreamSynchronize(st));
  std::vector<double> bb(nsys);
  for (int y = 0; y < nsys; ++y) {
    bb[y] = w->dscal_host[y];
    if (!(bb[y] < 1e300)) return set_error(WD_ERR_NONFINITE, "wd_solve: |b|^2 of system %d is not finite", y);
  }
  WD_TRY(blas_convert(G, WD_F64, vref(b, 2, sb), WD_F64, vref(x, 2, sb), 0.0, nullptr, nsys, st));
  WD_TRY(blas_convert(G, WD_F64, vref(b, 2, sb), WD_F64, vref(r64, 2, 2 * h64), 1.0, nullptr, nsys, st));
  std::vector<CgScalars> init(nsys);
  for (int y = 0; y < nsys; ++y) {
    init[y] = CgScalars{};
    init[y].rnorm2 = bb[y];
    init[y].bb = bb[y];
  }
  std::vector<double> rn2(bb);
  std::vector<int> active(nsys, 1), stalls(nsys, 0);
  std::vector<double> best(nsys, 1e300);
  int total_iters = 0;
  const int max_outer = 200;
  for (int outer = 0; outer < max_outer; ++outer) {
    int n_active = 0;
    for (int y = 0; y < nsys; ++y) {
      if (!active[y]) continue;
      if (bb[y] == 0.0 || rn2[y] <= tol * tol * bb[y]) active[y] = 0;
      else if (!(rn2[y] < 1e300)) active[y] = 0;
      else {
        if (rn2[y] < 0.5 * best[y]) { best[y] = rn2[y]; stalls[y] = 0; }
        else if (++stalls[y] >= 3) active[y] = 0;
      }
      n_active += active[y];
    }
    if (n_active == 0 || total_iters >= prm.max_iter) break;
    // rh32 = r / |r| (per-system scale from sc.rnorm2); systems already done
    // get a zero right-hand side and converge immediately.
    for (int y = 0; y < nsys; ++y) {
      init[y].rnorm2 = active[y] ? rn2[y] : 1.0;
      init[y].stop2 = active[y] ? prm.inner_tol * prm.inner_tol : 1e300;
      init[y].max_iters = std::max(1, prm.max_iter - total_iters);
      w->sc_host[y] = init[y];
    }
    WD_HIP(hipMemcpyAsync(w->sc, w->sc_host, sizeof(CgScalars) * nsys, hipMemcpyHostToDevice, st));
    WD_TRY(blas_convert(G, WD_F64, vref(r64, 2, 2 * h64), WD_F32, vref(rh32, 2, 2 * h32), 1.0, w->sc, nsys, st));
    for (int y = 0; y < nsys; ++y)
      if (!active[y])
        WD_TRY(blas_convert(G, WD_F32, vref(rh32 + 2 * h32 * y, 2), WD_F32, vref(rh32 + 2 * h32 * y, 2), 0.0,
                            nullptr, 1, st));
    // s = bh = rh_e + k H_eo rh_o, in FP32 then stored as S (staged in e32's odd half)
    {
      HopCall hc{rh32 + h32, e32 + h32, rh32, kappa, 0, 0, nullptr, nullptr};
      // per-system strides: the mrhs launcher takes rhs_stride from the field layout of
      // contiguous systems, so stage through a launcher that accepts an explicit stride
      MrhsArgs m;
      m.in = hc.in; m.out = hc.out; m.X = hc.X; m.a = kappa; m.parity = 0; m.nrhs = nsys;
      m.rhs_stride = 2 * h32;
      if (nsys == 1) {
        DslashArgs a;
        a.in = hc.in; a.out = hc.out; a.X = hc.X; a.a = kappa; a.parity = 0;
        WD_TRY(launch_dslash(g, WD_F32, a, st));
      } else {
        WD_TRY(launch_dslash_mrhs_ex(g, WD_F32, m, st));
      }
      WD_TRY(blas_convert(G, WD_F32, vref(e32 + h32, 1, 2 * h32), S, vref(V.s, 1, hS), 1.0, nullptr, nsys, st));
    }
    int calls = 1;
    WD_TRY(cgls_run(g, w, V, kappa, init.data(), prm, st, calls));
    int it_max = 0;
    for (int y = 0; y < nsys; ++y) {
      it_max = std::max(it_max, w->sc_host[y].iters);
      if (active[y]) infos[y].iters += w->sc_host[y].iters;
    }
    total_iters += it_max;
    // e_o = rh_o + k H_oe x_e   (FP32)
    {
      MrhsArgs m;
      m.in = e32; m.out = e32 + h32; m.X = rh32 + h32; m.a = kappa; m.parity = 1; m.nrhs = nsys;
      m.rhs_stride = 2 * h32;
      if (nsys == 1) {
        DslashArgs a;
        a.in = e32; a.out = e32 + h32; a.X = rh32 + h32; a.a = kappa; a.parity = 1;
        WD_TRY(launch_dslash(g, WD_F32, a, st));
      } else {
        WD_TRY(launch_dslash_mrhs_ex(g, WD_F32, m, st));
      }
    }
    calls += 1;
    // x += |r| e  (inactive systems have rnorm2 = 1 and e = 0)
    WD_TRY(blas_accum(G, WD_F32, vref(e32, 2, 2 * h32), vref(x, 2, sb), 1.0, w->sc, nsys, st));
    // r = b - D x, |r|^2
    WD_TRY(true_residual64(g, b, x, r64, nsys, sb, kappa, w->sc, red, st));
    calls += 2;
    WD_HIP(hipMemcpyAsync(w->sc_host, w->sc, sizeof(CgScalars) * nsys, hipMemcpyDeviceToHost, st));
    WD_HIP(hipStreamSynchronize(st));
    for (int y = 0; y < nsys; ++y) {
      if (!active[y]) continue;
      rn2[y] = w->sc_host[y].rnorm2;
      infos[y].outer_iters += 1;
      infos[y].dslash_calls += calls;
    }
  }
  wd_status worst = WD_OK;
  for (int y = 0; y < nsys; ++y) {
    infos[y].true_rel_resid = bb[y] > 0 ? sqrt(rn2[y] / bb[y]) : 0.0;
    infos[y].status = infos[y].true_rel_resid <= tol ? WD_OK : WD_NOT_CONVERGED;
    if (infos[y].status != WD_OK) worst = WD_NOT_CONVERGED;
  }
  return worst;
}

// ------------------------------------------------------------ entry points
static wd_status begin_solve(const wd_gauge *g, hipStream_t &st) {
  st = g->own_stream;
  hipEvent_t ev;
  WD_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  WD_HIP(hipEventRecord(ev, g->stream));
  WD_HIP(hipStreamWaitEvent(st, ev, 0));
  WD_HIP(hipEventDestroy(ev));
  return WD_OK;
}

wd_status solve(wd_gauge *g, const void *b, void *x, double kappa, double tol, const wd_solve_params &prm,
                wd_solve_info &info) {
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t st;
  WD_TRY(begin_solve(g, st));
  wd_status rc;
  if (prm.solver == WD_SOLVER_CG) {
    rc = solve_cg64(g, b, x, kappa, tol, prm, info, st);
  } else if (prm.solver == WD_SOLVER_DEFECT_CG) {
    rc = solve_defect(g, b, x, 1, 0, kappa, tol, prm, &info, st);
  } else if (prm.solver == WD_SOLVER_FGCR) {
    rc = solve_fgcr(g, b, x, kappa, tol, prm, info, st);
  } else if (prm.solver == WD_SOLVER_DEFECT_FGCR) {
    rc = solve_fgcr_mixed(g, b, x, kappa, tol, prm, info, st);
  } else if (prm.solver == WD_SOLVER_CGLS_FULL) {
    rc = solve_cgls_full64(g, b, x, kappa, tol, prm, info, st);
  } else {
    return set_error(WD_ERR_ARG, "wd_solve: unknown solver %d", prm.solver);
  }
  if (rc < 0) return rc;
  WD_HIP(hipStreamSynchronize(st));
  info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  info.status = rc;
  return rc;
}

wd_status solve_mrhs(wd_gauge *g, const void *b, void *x, int nrhs, double kappa, double tol,
                     const wd_solve_params &prm, wd_solve_info *infos) {
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t st;
  WD_TRY(begin_solve(g, st));
  const size_t sb = 2 * half_bytes(g->geom, WD_F64);
  wd_status rc = solve_defect(g, b, x, nrhs, sb, kappa, tol, prm, infos, st);
  if (rc < 0) return rc;
  WD_HIP(hipStreamSynchronize(st));
  const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int y = 0; y < nrhs; ++y) infos[y].seconds = sec;
  return rc;
}

}  // namespace wd
