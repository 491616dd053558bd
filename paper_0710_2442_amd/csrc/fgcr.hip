// Flexible GCR(m) on the full Wilson-Dirac operator with a right
// preconditioner (the PTC network, or the identity), FP64 vectors.
//
//   z_k = N(r);  w_k = D z_k;  modified Gram-Schmidt of w_k against the
//   stored w_j (the same combination applied to z_j);  normalise;
//   a = <w_k, r>;  x += a z_k;  r -= a w_k.
// After m directions the basis is dropped and r is recomputed as b - D x in
// FP64.  If |r| has not fallen below 0.99 of its best value within
// `stagnation` iterations, or stops being finite, the solve falls back to
// plain FP64 even-odd CG on the remaining residual (x += D^{-1} r), which is
// also what decides convergence: every exit reports the FP64 true residual.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "wd_blas.h"
#include "wd_ptc.h"
#include "wd_solver.h"

namespace wd {

namespace {

struct Buf {
  void *p = nullptr;
  ~Buf() {
    if (p) (void)hipFree(p);
  }
};

struct FgcrCtx {
  wd_gauge *g;
  hipStream_t st;
  RedBuf red;
  double *dres;   // device results of reductions
  double *hres;   // pinned host copy
  int dslash_calls = 0;
};

wd_status sync_read(FgcrCtx &c, int n, double *out) {
  WD_HIP(hipMemcpyAsync(c.hres, c.dres, sizeof(double) * n, hipMemcpyDeviceToHost, c.st));
  WD_HIP(hipStreamSynchronize(c.st));
  for (int i = 0; i < n; ++i) out[i] = c.hres[i];
  return WD_OK;
}

wd_status dot(FgcrCtx &c, const void *a, const void *b, double &re, double &im) {
  WD_TRY(blas_cdot(c.g->geom, WD_F64, vref(a, 2), vref(b, 2), 1, c.red, c.dres, c.st));
  double v[2];
  WD_TRY(sync_read(c, 2, v));
  re = v[0];
  im = v[1];
  return WD_OK;
}

wd_status nrm2(FgcrCtx &c, const void *a, double &out) {
  WD_TRY(blas_norm2(c.g->geom, WD_F64, vref(a, 2), 1, c.red, c.dres, c.st));
  return sync_read(c, 1, &out);
}

// y += (cre + i cim) x
wd_status axpy(FgcrCtx &c, double cre, double cim, const void *x, void *y) {
  return blas_caxpy(c.g->geom, WD_F64, cre, cim, vref(x, 2), vref(y, 2), 1, c.st);
}

wd_status scale(FgcrCtx &c, void *x, double s) {
  return blas_convert(c.g->geom, WD_F64, vref(x, 2), WD_F64, vref(x, 2), s, nullptr, 1, c.st);
}

// out = D_W in (FP64 full fields)
wd_status apply_D(FgcrCtx &c, const void *in, void *out, double kappa) {
  const size_t hb = half_bytes(c.g->geom, WD_F64);
  for (int p = 0; p < 2; ++p) {
    DslashArgs a;
    a.in = (const char *)in + (1 - p) * hb;
    a.out = (char *)out + p * hb;
    a.X = (const char *)in + p * hb;
    a.a = -kappa;
    a.parity = p;
    WD_TRY(launch_dslash(c.g, WD_F64, a, c.st));
  }
  c.dslash_calls += 2;
  return WD_OK;
}

}  // namespace

wd_status solve_fgcr(wd_gauge *g, const void *b, void *x, double kappa, double tol, const wd_solve_params &prm,
                     wd_solve_info &info, hipStream_t st) {
  const wd_ptc *N = prm.precond;
  if (N && ptc_gauge(N) != g)
    return set_error(WD_ERR_ARG, "FGCR: the preconditioner was created on another gauge handle");
  const Geom &G = g->geom;
  const int m = prm.fgcr_m;
  const size_t f64 = 2 * half_bytes(G, WD_F64), f32 = 2 * half_bytes(G, WD_F32);
  // r, e, Z[m], W[m] in FP64; two FP32 fields for the network
  Buf mem, red, pin;
  const size_t nred = (size_t)std::max<unsigned>(dslash_grid_blocks(g), BLAS_MAX_BLOCKS) * 2 + 256;
  WD_HIP(hipMalloc(&mem.p, f64 * (2 + 2 * (size_t)m) + 2 * f32));
  WD_HIP(hipMalloc(&red.p, nred * sizeof(double) + 256));
  WD_HIP(hipMemsetAsync((char *)red.p + nred * sizeof(double), 0, 256, st));
  double *hres = nullptr;
  WD_HIP(hipHostMalloc((void **)&hres, 64 * sizeof(double), hipHostMallocDefault));
  struct HostFree {
    double *p;
    ~HostFree() { (void)hipHostFree(p); }
  } hf{hres};
  char *c0 = (char *)mem.p;
  void *r = c0, *e = c0 + f64;
  std::vector<void *> Z(m), W(m);
  for (int k = 0; k < m; ++k) {
    Z[k] = c0 + (2 + k) * f64;
    W[k] = c0 + (2 + m + k) * f64;
  }
  void *t_in = c0 + (2 + 2 * (size_t)m) * f64, *t_out = (char *)t_in + f32;
  FgcrCtx c;
  c.g = g;
  c.st = st;
  c.dres = (double *)red.p;
  c.red = RedBuf{(double *)red.p + 64, (unsigned *)((char *)red.p + nred * sizeof(double))};
  c.hres = hres;

  double bb;
  WD_TRY(nrm2(c, b, bb));
  if (!(bb < 1e300)) return set_error(WD_ERR_NONFINITE, "FGCR: |b|^2 is not finite");
  WD_TRY(blas_convert(G, WD_F64, vref(b, 2), WD_F64, vref(x, 2), 0.0, nullptr, 1, st));  // x = 0
  if (bb == 0.0) {
    info.true_rel_resid = 0.0;
    return WD_OK;
  }
  const double bn = sqrt(bb);
  WD_TRY(blas_convert(G, WD_F64, vref(b, 2), WD_F64, vref(r, 2), 1.0, nullptr, 1, st));
  double rn = bn, best = 1e300;
  int since_best = 0, it = 0;
  const int stagnation = 30;
  bool converged = false, fallback = false;
  while (it < prm.max_iter && !converged && !fallback) {
    int k = 0;
    for (; k < m && it < prm.max_iter; ++k) {
      // z = N(r / |r|) (the network is linear; the scaling keeps the FP32/BF16 range)
      if (N) {
        WD_TRY(blas_convert(G, WD_F64, vref(r, 2), WD_F32, vref(t_in, 2), 1.0 / rn, nullptr, 1, st));
        WD_TRY(ptc_apply(N, t_in, t_out, st));
        WD_TRY(blas_convert(G, WD_F32, vref(t_out, 2), WD_F64, vref(Z[k], 2), 1.0, nullptr, 1, st));
      } else {
        WD_TRY(blas_convert(G, WD_F64, vref(r, 2), WD_F64, vref(Z[k], 2), 1.0 / rn, nullptr, 1, st));
      }
      WD_TRY(apply_D(c, Z[k], W[k], kappa));
      for (int j = 0; j < k; ++j) {
        double cre, cim;
        WD_TRY(dot(c, W[j], W[k], cre, cim));
        WD_TRY(axpy(c, -cre, -cim, W[j], W[k]));
        WD_TRY(axpy(c, -cre, -cim, Z[j], Z[k]));
      }
      double ww;
      WD_TRY(nrm2(c, W[k], ww));
      ++it;
      if (!(ww > 0.0) || !(ww < 1e300)) {
        fallback = true;
        break;
      }
      const double inv = 1.0 / sqrt(ww);
      WD_TRY(scale(c, W[k], inv));
      WD_TRY(scale(c, Z[k], inv));
      double are, aim;
      WD_TRY(dot(c, W[k], r, are, aim));
      WD_TRY(axpy(c, are, aim, Z[k], x));
      WD_TRY(axpy(c, -are, -aim, W[k], r));
      double rr;
      WD_TRY(nrm2(c, r, rr));
      rn = sqrt(rr);
      if (!(rn < 1e300)) {
        fallback = true;
        break;
      }
      if (rn < 0.99 * best) {
        best = rn;
        since_best = 0;
      } else if (++since_best >= stagnation) {
        fallback = true;
        break;
      }
      if (rn <= tol * bn) break;
    }
    // restart (and convergence check) with the FP64 true residual
    WD_TRY(apply_D(c, x, e, kappa));
    WD_TRY(blas_convert(G, WD_F64, vref(b, 2), WD_F64, vref(r, 2), 1.0, nullptr, 1, st));
    WD_TRY(axpy(c, -1.0, 0.0, e, r));
    double rr;
    WD_TRY(nrm2(c, r, rr));
    rn = sqrt(rr);
    info.outer_iters += 1;
    if (!(rn < 1e300)) fallback = true;
    if (rn <= tol * bn) converged = true;
  }
  info.iters = it;
  info.dslash_calls = c.dslash_calls;
  if (!converged && (fallback || it >= prm.max_iter)) {
    // plain FP64 CG on the remaining residual: x <- x + D^{-1} r
    wd_solve_params cg = prm;
    cg.solver = WD_SOLVER_CG;
    wd_solve_info ci;
    memset(&ci, 0, sizeof ci);
    if (!(rn < 1e300)) {  // restart from x = 0 if x itself went bad
      WD_TRY(blas_convert(G, WD_F64, vref(b, 2), WD_F64, vref(x, 2), 0.0, nullptr, 1, st));
      WD_TRY(blas_convert(G, WD_F64, vref(b, 2), WD_F64, vref(r, 2), 1.0, nullptr, 1, st));
      rn = bn;
    }
    const double tol_r = std::max(1e-15, tol * bn / rn);
    wd_status rc = solve_cg64(g, r, e, kappa, 0.5 * tol_r, cg, ci, st);
    if (rc < 0) return rc;
    WD_TRY(axpy(c, 1.0, 0.0, e, x));
    info.iters += ci.iters;
    info.dslash_calls += ci.dslash_calls;
    info.fallback_used = 1;
    WD_TRY(apply_D(c, x, e, kappa));
    WD_TRY(blas_convert(G, WD_F64, vref(b, 2), WD_F64, vref(r, 2), 1.0, nullptr, 1, st));
    WD_TRY(axpy(c, -1.0, 0.0, e, r));
    double rr;
    WD_TRY(nrm2(c, r, rr));
    rn = sqrt(rr);
  }
  info.true_rel_resid = rn / bn;
  return info.true_rel_resid <= tol ? WD_OK : WD_NOT_CONVERGED;
}

}  // namespace wd
