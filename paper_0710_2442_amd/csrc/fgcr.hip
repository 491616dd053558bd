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
#include <utility>
#include <vector>

#include "wd_blas.h"
#include "wd_device.h"
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

// out = D_W in (FP64 full fields): the one-launch marching kernel where it
// fills the device, else one hop per parity
wd_status apply_D(FgcrCtx &c, const void *in, void *out, double kappa) {
  c.dslash_calls += 2;
  if (dirac_fills_device(c.g, WD_F64)) {
    DiracArgs a;
    a.in = in;
    a.out = out;
    a.X = in;
    a.a = -kappa;
    return launch_dirac(c.g, WD_F64, a, c.st);
  }
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
  c.red = RedBuf{(double *)red.p + 64};
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

// ------------------------------------------------------------------------
// Mixed precision: FP64 defect correction around an FP32 even-odd FGCR.
//
// Outer (FP64): r = b - D x;  rh = r / |r| (FP32);  Schur right-hand side
// s = rh_e + kappa H_eo rh_o;  inner solve of Mhat e_e = s with
// Mhat = 1 - kappa^2 H_eo H_oe to |s - Mhat e_e| <= inner_tol |s|;
// e_o = rh_o + kappa H_oe e_e;  x += |r| e;  repeat until the FP64 true
// residual meets tol.
//
// Inner (FP32 vectors, FP64 reductions), one direction per iteration:
//   z_k = [N (r, 0)]_e   (the network restricted to the even sites, on the
//                         matrix cores when its activations are BF16; z = r
//                         without a network)
//   w_k = Mhat z_k
//   c_j = <w_j, w_k> / |w_j|^2 (j < k, one fused pass: classical Gram-Schmidt
//         against an unnormalised basis)
//   w_k -= sum c_j w_j,  z_k -= sum c_j z_j,  sigma_k = |w_k|^2,
//   rho = <w_k, r>       (one fused pass)
//   alpha = rho / sigma_k,  e += alpha z_k,  r -= alpha w_k,  |r|^2 (one pass)
// The basis is dropped after m directions (restart).  All coefficients stay
// in device memory; the host reads |r|^2 once per iteration.

namespace {

constexpr int FG_MMAX = 16;
constexpr int FG_BS = 256;
constexpr unsigned FG_MAX_BLOCKS = 2048;

struct KFg {
  int vh;
  unsigned nblk;
  const char *W[FG_MMAX];  // basis w_j (half fields, storage precision S)
  const char *Z[FG_MMAX];  // and z_j
  char *wk, *zk;           // the new direction (updated in place; S)
  char *r;                 // residual (S)
  char *e;                 // solution (FP32)
  double *dots;    // [2 FG_MMAX]: <w_j, w_k>
  double *sig;     // [FG_MMAX]: |w_j|^2
  double *rho;     // [2]: <w_k, r>
  double *rr;      // |r|^2
  float *alpha;    // [2 FG_MMAX]: the step lengths of the current cycle (re, im)
  int k;
  double *partials;
};

using F4 = Spinor<WD_F32>;

// <a, b> = sum conj(a) b over one site, in FP64
__device__ __forceinline__ void site_dot(const cplx<float> (&a)[12], const cplx<float> (&b)[12], double &re,
                                         double &im) {
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    re += (double)a[c].re * b[c].re + (double)a[c].im * b[c].im;
    im += (double)a[c].re * b[c].im - (double)a[c].im * b[c].re;
  }
}

template <int S, int K>
__global__ __launch_bounds__(FG_BS) void k_fg_dots(KFg a) {
  using V = Spinor<S>;
  double acc[2 * K];
#pragma unroll
  for (int j = 0; j < 2 * K; ++j) acc[j] = 0.0;
  for (long i = (long)blockIdx.x * FG_BS + threadIdx.x; i < a.vh; i += (long)a.nblk * FG_BS) {
    cplx<float> w[12];
    V::load(a.wk, i, w);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      cplx<float> v[12];
      V::load(a.W[j], i, v);
      site_dot(v, w, acc[2 * j], acc[2 * j + 1]);
    }
  }
  block_sum_store<2 * K>(acc, a.partials, a.nblk, blockIdx.x);
}

template <int S, int K>
__global__ __launch_bounds__(FG_BS) void k_fg_orth(KFg a) {
  using V = Spinor<S>;
  cplx<float> c[K > 0 ? K : 1];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const double s = a.sig[j];
    const double f = (s > 0.0) ? 1.0 / s : 0.0;
    c[j] = {(float)(a.dots[2 * j] * f), (float)(a.dots[2 * j + 1] * f)};
  }
  double acc[3] = {0.0, 0.0, 0.0};
  for (long i = (long)blockIdx.x * FG_BS + threadIdx.x; i < a.vh; i += (long)a.nblk * FG_BS) {
    cplx<float> w[12], z[12];
    V::load(a.wk, i, w);
    if constexpr (K > 0) {
      V::load(a.zk, i, z);
#pragma unroll
      for (int j = 0; j < K; ++j) {
        cplx<float> v[12];
        const cplx<float> m = {-c[j].re, -c[j].im};
        V::load(a.W[j], i, v);
#pragma unroll
        for (int q = 0; q < 12; ++q) cfma(w[q], m, v[q]);
        V::load(a.Z[j], i, v);
#pragma unroll
        for (int q = 0; q < 12; ++q) cfma(z[q], m, v[q]);
      }
      V::template store<false>(a.wk, i, w);
      V::template store<false>(a.zk, i, z);
      // the norms and products below see the stored (rounded) direction
      if constexpr (S != WD_F32) V::load(a.wk, i, w);
    }
    cplx<float> r[12];
    V::load(a.r, i, r);
#pragma unroll
    for (int q = 0; q < 12; ++q) acc[0] += (double)w[q].re * w[q].re + (double)w[q].im * w[q].im;
    site_dot(w, r, acc[1], acc[2]);
  }
  block_sum_store<3>(acc, a.partials, a.nblk, blockIdx.x);
}

// r -= alpha w_k, |r|^2; alpha_k is kept for the solution update, which is
// applied once per restart cycle (k_fg_accum)
template <int S>
__global__ __launch_bounds__(FG_BS) void k_fg_step(KFg a) {
  using V = Spinor<S>;
  const double s = a.sig[a.k];
  const bool ok = s > 0.0 && s < 1e300;
  const cplx<float> al = {ok ? (float)(a.rho[0] / s) : 0.f, ok ? (float)(a.rho[1] / s) : 0.f};
  const cplx<float> ml = {-al.re, -al.im};
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.alpha[2 * a.k] = al.re;
    a.alpha[2 * a.k + 1] = al.im;
  }
  double acc[1] = {0.0};
  for (long i = (long)blockIdx.x * FG_BS + threadIdx.x; i < a.vh; i += (long)a.nblk * FG_BS) {
    cplx<float> w[12], r[12];
    V::load(a.wk, i, w);
    V::load(a.r, i, r);
#pragma unroll
    for (int q = 0; q < 12; ++q) cfma(r[q], ml, w[q]);
    V::template store<false>(a.r, i, r);
    if constexpr (S != WD_F32) V::load(a.r, i, r);  // |r|^2 of the stored residual
#pragma unroll
    for (int q = 0; q < 12; ++q) acc[0] += (double)r[q].re * r[q].re + (double)r[q].im * r[q].im;
  }
  block_sum_store<1>(acc, a.partials, a.nblk, blockIdx.x);
}

// e += sum_{j < K} alpha_j z_j for the K steps of a cycle, in step order
// (the same FP32 operations, in the same order, as updating e at every step)
template <int S, int K>
__global__ __launch_bounds__(FG_BS) void k_fg_accum(KFg a) {
  using V = Spinor<S>;
  cplx<float> al[K];
#pragma unroll
  for (int j = 0; j < K; ++j) al[j] = {a.alpha[2 * j], a.alpha[2 * j + 1]};
  for (long i = (long)blockIdx.x * FG_BS + threadIdx.x; i < a.vh; i += (long)a.nblk * FG_BS) {
    cplx<float> e[12];
    F4::load(a.e, i, e);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      cplx<float> z[12];
      V::load(a.Z[j], i, z);
#pragma unroll
      for (int q = 0; q < 12; ++q) cfma(e[q], al[j], z[q]);
    }
    F4::store<false>(a.e, i, e);
  }
}

// Second stage of the three kernels above: value j = sum of the block
// partials (block order) goes to dst[j] (dots, or rr), or for the
// orthogonalisation to sig[k] (j = 0) and rho (j = 1, 2).
constexpr int FG_FIN = 1024;
__global__ __launch_bounds__(FG_FIN) void k_fg_finish(KFg a, int which) {
  const int j = blockIdx.x;
  double v[1] = {0.0};
  for (unsigned b = threadIdx.x; b < a.nblk; b += FG_FIN) v[0] += a.partials[(size_t)j * a.nblk + b];
  block_sum_n<1>(v);
  if (threadIdx.x != 0) return;
  if (which == 0) a.dots[j] = v[0];
  else if (which == 1) (j == 0 ? a.sig[a.k] : a.rho[j - 1]) = v[0];
  else *a.rr = v[0];
}

template <int S, int K>
void launch_dots_k(const KFg &a, hipStream_t st) {
  hipLaunchKernelGGL((k_fg_dots<S, K>), dim3(a.nblk), dim3(FG_BS), 0, st, a);
}
template <int S, int K>
void launch_orth_k(const KFg &a, hipStream_t st) {
  hipLaunchKernelGGL((k_fg_orth<S, K>), dim3(a.nblk), dim3(FG_BS), 0, st, a);
}

template <int S, int... Ks>
void launch_dots(const KFg &a, int k, hipStream_t st, std::integer_sequence<int, Ks...>) {
  ((k == Ks + 1 ? launch_dots_k<S, Ks + 1>(a, st) : void()), ...);
}
template <int S, int... Ks>
void launch_orth(const KFg &a, int k, hipStream_t st, std::integer_sequence<int, Ks...>) {
  ((k == Ks ? launch_orth_k<S, Ks>(a, st) : void()), ...);
}

template <int S, int K>
void launch_accum_k(const KFg &a, hipStream_t st) {
  hipLaunchKernelGGL((k_fg_accum<S, K>), dim3(a.nblk), dim3(FG_BS), 0, st, a);
}
template <int S, int... Ks>
void launch_accum(const KFg &a, int K, hipStream_t st, std::integer_sequence<int, Ks...>) {
  ((K == Ks + 1 ? launch_accum_k<S, Ks + 1>(a, st) : void()), ...);
}

// One FGCR direction after w_k = Mhat z_k: orthogonalise against the k
// earlier directions, then the step; FP32 arithmetic on S-stored vectors.
template <int S>
void fg_direction(const KFg &a, int k, hipStream_t st) {
  if (k > 0) {
    launch_dots<S>(a, k, st, std::make_integer_sequence<int, FG_MMAX - 1>{});
    hipLaunchKernelGGL(k_fg_finish, dim3(2 * k), dim3(FG_FIN), 0, st, a, 0);
  }
  launch_orth<S>(a, k, st, std::make_integer_sequence<int, FG_MMAX>{});
  hipLaunchKernelGGL(k_fg_finish, dim3(3), dim3(FG_FIN), 0, st, a, 1);
  hipLaunchKernelGGL(k_fg_step<S>, dim3(a.nblk), dim3(FG_BS), 0, st, a);
  hipLaunchKernelGGL(k_fg_finish, dim3(1), dim3(FG_FIN), 0, st, a, 2);
}

// out = Mhat in = in - kappa^2 H_eo H_oe in   (even half fields in precision
// S, FP32 arithmetic; tmp: odd half)
wd_status apply_mhat(wd_gauge *g, wd_prec S, const void *in, void *out, void *tmp, double kappa, hipStream_t st) {
  DslashArgs a;
  a.in = in;
  a.out = tmp;
  a.a = 1.0;
  a.parity = 1;
  WD_TRY(launch_dslash(g, S, a, st));
  DslashArgs b;
  b.in = tmp;
  b.out = out;
  b.X = in;
  b.a = -kappa * kappa;
  b.parity = 0;
  return launch_dslash(g, S, b, st);
}

}  // namespace

wd_status solve_fgcr_mixed(wd_gauge *g, const void *b, void *x, double kappa, double tol,
                           const wd_solve_params &prm, wd_solve_info &info, hipStream_t st) {
  const wd_ptc *N = prm.precond;
  if (N && ptc_gauge(N) != g)
    return set_error(WD_ERR_ARG, "FGCR: the preconditioner was created on another gauge handle");
  const int m = std::min(prm.fgcr_m, FG_MMAX);
  const Geom &G = g->geom;
  const wd_prec S = prm.inner_prec;  // storage of R, T, Z, W (FP32 or BF16)
  if (S != WD_F32 && S != WD_BF16) return set_error(WD_ERR_PREC, "FGCR: inner_prec must be FP32 or BF16");
  const size_t h64 = half_bytes(G, WD_F64), h32 = half_bytes(G, WD_F32), hS = half_bytes(G, S);
  // r64, d64 (2 h64 each); rh, e (2 h32 each); R, T, Z[m], W[m] (hS each); then the
  // device scalars ([0, 128) CgScalars, [128, 536) dots/sig/rho/rr, [640, 768) the cycle's
  // step lengths) and the reduction partials.  Kept in the handle between solves (grown
  // when a solve needs more).
  const unsigned nblk = (unsigned)std::min<long>(std::max<long>(1, ((long)G.vh + FG_BS - 1) / FG_BS), FG_MAX_BLOCKS);
  const size_t npart = std::max<size_t>((size_t)2 * FG_MMAX * nblk,
                                        (size_t)2 * std::max<unsigned>(dslash_grid_blocks(g), BLAS_MAX_BLOCKS));
  const size_t vec_bytes = round_up(4 * h64 + 4 * h32 + (2 + 2 * (size_t)m) * hS, 256);
  const size_t scal_bytes = 1024;
  const size_t need = vec_bytes + scal_bytes + npart * sizeof(double);
  if (!g->fg_mem || g->fg_bytes < need) {
    if (g->fg_mem) {
      WD_HIP(hipStreamSynchronize(st));
      WD_HIP(hipFree(g->fg_mem));
      g->fg_mem = nullptr;
      g->fg_bytes = 0;
    }
    if (hipMalloc(&g->fg_mem, need) != hipSuccess) {
      (void)hipGetLastError();
      g->fg_mem = nullptr;
      return set_error(WD_ERR_OOM, "FGCR: cannot allocate %zu bytes", need);
    }
    g->fg_bytes = need;
  }
  if (!g->fg_host) WD_HIP(hipHostMalloc((void **)&g->fg_host, 64 * sizeof(double), hipHostMallocDefault));
  double *hres = g->fg_host;
  char *red = (char *)g->fg_mem + vec_bytes;
  WD_HIP(hipMemsetAsync(red, 0, scal_bytes, st));
  char *c0 = (char *)g->fg_mem;
  char *r64 = c0, *d64 = c0 + 2 * h64, *rh = c0 + 4 * h64, *e32 = rh + 2 * h32;
  char *R = e32 + 2 * h32, *T = R + hS;
  char *E = e32;  // inner solution = even half of e32 (FP32)
  KFg a{};
  a.vh = G.vh;
  a.nblk = nblk;
  for (int k = 0; k < m; ++k) {
    a.Z[k] = T + (1 + (size_t)k) * hS;
    a.W[k] = T + (1 + (size_t)m + k) * hS;
  }
  CgScalars *sc = (CgScalars *)red;
  double *ds = (double *)(red + 128);
  a.dots = ds;
  a.sig = ds + 2 * FG_MMAX;
  a.rho = a.sig + FG_MMAX;
  a.rr = a.rho + 2;
  a.alpha = (float *)(red + 640);  // 2 FG_MMAX floats inside the scalar block
  static_assert(sizeof(CgScalars) <= 128, "CgScalars exceed their slot");
  static_assert(128 + (2 * FG_MMAX + FG_MMAX + 3) * sizeof(double) <= 640, "FGCR scalars overlap");
  static_assert(640 + 2 * FG_MMAX * sizeof(float) <= 1024, "FGCR step lengths exceed the scalar block");
  a.r = R;
  a.e = E;
  a.partials = (double *)(red + scal_bytes);
  RedBuf rb{a.partials};
  auto accum = [&](int K) {
    if (S == WD_F32) launch_accum<WD_F32>(a, K, st, std::make_integer_sequence<int, FG_MMAX>{});
    else launch_accum<WD_BF16>(a, K, st, std::make_integer_sequence<int, FG_MMAX>{});
  };
  auto read = [&](const double *dev, int n, double *out) -> wd_status {
    WD_HIP(hipMemcpyAsync(hres, dev, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    WD_HIP(hipStreamSynchronize(st));
    for (int q = 0; q < n; ++q) out[q] = hres[q];
    return WD_OK;
  };

  // |b|^2;  x = 0;  r = b
  double bb;
  WD_TRY(blas_norm2(G, WD_F64, vref(b, 2), 1, rb, a.rr, st));
  WD_TRY(read(a.rr, 1, &bb));
  if (!(bb < 1e300)) return set_error(WD_ERR_NONFINITE, "FGCR: |b|^2 is not finite");
  WD_TRY(blas_convert(G, WD_F64, vref(b, 2), WD_F64, vref(x, 2), 0.0, nullptr, 1, st));
  if (bb == 0.0) {
    info.true_rel_resid = 0.0;
    return WD_OK;
  }
  WD_TRY(blas_convert(G, WD_F64, vref(b, 2), WD_F64, vref(r64, 2), 1.0, nullptr, 1, st));
  {
    CgScalars h{};
    h.rnorm2 = bb;
    h.bb = bb;
    WD_HIP(hipMemcpyAsync(sc, &h, sizeof h, hipMemcpyHostToDevice, st));
    WD_HIP(hipStreamSynchronize(st));
  }
  double rn2 = bb, best_outer = 1e300;
  int stalls = 0, it = 0, calls = 0;
  bool converged = false, fallback = false;
  const int stagnation = 30;
  for (int outer = 0; outer < 100 && !fallback; ++outer) {
    if (rn2 <= tol * tol * bb) {
      converged = true;
      break;
    }
    if (!(rn2 < 1e300) || it >= prm.max_iter) {
      fallback = true;
      break;
    }
    if (rn2 < 0.5 * best_outer) {
      best_outer = rn2;
      stalls = 0;
    } else if (++stalls >= 3) {
      fallback = true;
      break;
    }
    // rh = r / |r|;  R = rh_e + kappa H_eo rh_o;  E = 0
    WD_TRY(blas_convert(G, WD_F64, vref(r64, 2), WD_F32, vref(rh, 2), 1.0, sc, 1, st));
    {
      // FP32, staged in e32's odd half when R is stored in lower precision
      DslashArgs d;
      d.in = rh + h32;
      d.out = (S == WD_F32) ? R : e32 + h32;
      d.X = rh;
      d.a = kappa;
      d.parity = 0;
      WD_TRY(launch_dslash(g, WD_F32, d, st));
      if (S != WD_F32) WD_TRY(blas_convert(G, WD_F32, vref(e32 + h32, 1), S, vref(R, 1), 1.0, nullptr, 1, st));
      calls += 1;
    }
    WD_HIP(hipMemsetAsync(E, 0, h32, st));
    double s2;
    WD_TRY(blas_norm2(G, S, vref(R, 1), 1, rb, a.rr, st));
    WD_TRY(read(a.rr, 1, &s2));
    const double target = prm.inner_tol * prm.inner_tol * s2;
    double rr = s2, best = s2;
    int since = 0, k = 0;
    while (rr > target && it < prm.max_iter) {
      char *zk = (char *)a.Z[k], *wk = (char *)a.W[k];
      if (N && ptc_act(N) == WD_BF16) WD_TRY(ptc_apply_even_b(N, R, S, zk, S, st));
      else if (N) WD_TRY(ptc_apply_even(N, R, S, zk, S, st));
      else WD_TRY(blas_convert(G, S, vref(R, 1), S, vref(zk, 1), 1.0, nullptr, 1, st));
      WD_TRY(apply_mhat(g, S, zk, wk, T, kappa, st));
      calls += 2;
      a.wk = wk;
      a.zk = zk;
      a.k = k;
      if (S == WD_F32) fg_direction<WD_F32>(a, k, st);
      else fg_direction<WD_BF16>(a, k, st);
      WD_TRY(hip_check(hipGetLastError(), "fgcr launch"));
      WD_TRY(read(a.rr, 1, &rr));
      ++it;
      if (!(rr < 1e300)) {
        fallback = true;
        break;
      }
      if (rr < 0.98 * best) {
        best = rr;
        since = 0;
      } else if (++since >= stagnation) {
        fallback = true;
        break;
      }
      // the cycle's steps enter the solution when the basis wraps (and after the loop)
      k = k + 1;
      if (k == m) {
        accum(k);
        k = 0;
      }
    }
    if (fallback) break;
    if (k > 0) accum(k);
    // e_o = rh_o + kappa H_oe E;  x += |r| e;  r = b - D x
    {
      DslashArgs d;
      d.in = E;
      d.out = e32 + h32;
      d.X = rh + h32;
      d.a = kappa;
      d.parity = 1;
      WD_TRY(launch_dslash(g, WD_F32, d, st));
    }
    WD_TRY(blas_accum(G, WD_F32, vref(e32, 2), vref(x, 2), 1.0, sc, 1, st));
    WD_TRY(true_residual64(g, b, x, r64, 1, 0, kappa, sc, rb, st));
    calls += 3;
    WD_TRY(read(&sc->rnorm2, 1, &rn2));
    info.outer_iters += 1;
  }
  info.iters = it;
  info.dslash_calls = calls;
  if (!converged) {
    // plain FP64 CG on the remaining residual: x <- x + D^{-1} r
    if (!(rn2 < 1e300)) {  // restart from x = 0 if x itself went bad
      WD_TRY(blas_convert(G, WD_F64, vref(b, 2), WD_F64, vref(x, 2), 0.0, nullptr, 1, st));
      WD_TRY(blas_convert(G, WD_F64, vref(b, 2), WD_F64, vref(r64, 2), 1.0, nullptr, 1, st));
      rn2 = bb;
    }
    wd_solve_params cg = prm;
    cg.solver = WD_SOLVER_CG;
    wd_solve_info ci;
    memset(&ci, 0, sizeof ci);
    const double tol_r = std::max(1e-15, tol * sqrt(bb / rn2));
    wd_status rc = solve_cg64(g, r64, d64, kappa, 0.5 * tol_r, cg, ci, st);
    if (rc < 0) return rc;
    WD_TRY(blas_caxpy(G, WD_F64, 1.0, 0.0, vref(d64, 2), vref(x, 2), 1, st));
    info.iters += ci.iters;
    info.dslash_calls += ci.dslash_calls + 2;
    info.fallback_used = 1;
    WD_TRY(true_residual64(g, b, x, r64, 1, 0, kappa, sc, rb, st));
    WD_TRY(read(&sc->rnorm2, 1, &rn2));
  }
  info.true_rel_resid = sqrt(rn2 / bb);
  return info.true_rel_resid <= tol ? WD_OK : WD_NOT_CONVERGED;
}

void fgcr_free(wd_gauge *g) {
  if (g->fg_mem) (void)hipFree(g->fg_mem);
  if (g->fg_host) (void)hipHostFree(g->fg_host);
  g->fg_mem = nullptr;
  g->fg_host = nullptr;
  g->fg_bytes = 0;
}

}  // namespace wd
