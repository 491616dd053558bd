// Level-1 kernels on spin-colour fields: caxpy (Sec. 4), inner products and
// norms with FP64 accumulation in a fixed order, precision conversion, and
// the fused CG recurrences whose scalars never leave the device.
//
// Every kernel works on `nsys` independent systems at once (grid.y): system
// y's vectors start at y * sys_stride bytes and it owns its own scalar block
// and reduction slots, so a batch of right-hand sides shares each launch.
// A vector is `nhalf` half fields of vh valid sites (half_stride bytes apart).
#include "wd_blas.h"
#include "wd_device.h"

namespace wd {

template <int P>
using RealOf = typename Spinor<P>::real;

constexpr int BLAS_BS = 256;

struct VecGeom {
  int vh;
  int vpad;
  int nhalf;
  size_t half_stride;  // bytes between half fields of one vector (per precision)
};

struct KBlas {
  VecGeom v;
  unsigned nblk;  // blocks per system (grid.x)
  // operands (system 0); per-system offsets below
  const char *x;
  const char *y;
  char *out;
  char *out2;
  size_t sx, sy, so, so2;  // per-system byte strides of x, y, out, out2
  size_t hx, hy, ho, ho2;  // per-half byte strides
  double c_re, c_im;
  CgScalars *sc;
  int j;  // ping-pong slot of the CG iteration
  double *partials;
  double *result;  // reductions: per-system result (N doubles each)
};

__device__ __forceinline__ bool site_of(const VecGeom &v, long f, int &h, int &i) {
  h = (int)(f / v.vh);
  i = (int)(f - (long)h * v.vh);
  return h < v.nhalf;
}

// ------------------------------------------------------------ reductions
// A spinor read with streaming (non-temporal) loads, for operands read once
// per kernel (caxpy and the reductions |x|^2, <x, y>): full fields of the
// solvers are larger than the caches, so keeping them buys nothing and
// streaming them frees the caches for the hop's gathers.  FP16 and BF16 as
// Spinor<P>::load.
template <int P>
__device__ __forceinline__ void load_stream(const char *base, int i, cplx<RealOf<P>> (&s)[12]) {
  if constexpr (P == WD_F64) {
    const v2d *p = (const v2d *)base + chunk_base<Spinor<WD_F64>::CHUNK>((size_t)i);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const v2d v = ld_stream(p + 64 * c);
      s[c] = {v.x, v.y};
    }
  } else if constexpr (P == WD_F32) {
    const v4f *p = (const v4f *)base + chunk_base<Spinor<WD_F32>::CHUNK>((size_t)i);
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const v4f v = ld_stream(p + 64 * q);
      s[2 * q] = {v.x, v.y};
      s[2 * q + 1] = {v.z, v.w};
    }
  } else {
    Spinor<P>::load(base, (size_t)i, s);
  }
}

template <int P>
__global__ __launch_bounds__(BLAS_BS) void k_norm2(KBlas k) {
  using T = RealOf<P>;
  const int sys = blockIdx.y;
  const char *x = k.x + sys * k.sx;
  const long n = (long)k.v.vh * k.v.nhalf;
  double acc = 0.0;
  for (long f = (long)blockIdx.x * BLAS_BS + threadIdx.x; f < n; f += (long)k.nblk * BLAS_BS) {
    int h, i;
    site_of(k.v, f, h, i);
    cplx<T> a[12];
    load_stream<P>(x + h * k.hx, i, a);
#pragma unroll
    for (int c = 0; c < 12; ++c) acc += (double)a[c].re * a[c].re + (double)a[c].im * a[c].im;
  }
  double v[1] = {acc};
  block_sum_store<1>(v, k.partials + (size_t)sys * k.nblk, k.nblk, blockIdx.x);
}

template <int P>
__global__ __launch_bounds__(BLAS_BS) void k_cdot(KBlas k) {
  using T = RealOf<P>;
  const int sys = blockIdx.y;
  const char *x = k.x + sys * k.sx;
  const char *y = k.y + sys * k.sy;
  const long n = (long)k.v.vh * k.v.nhalf;
  double re = 0.0, im = 0.0;
  for (long f = (long)blockIdx.x * BLAS_BS + threadIdx.x; f < n; f += (long)k.nblk * BLAS_BS) {
    int h, i;
    site_of(k.v, f, h, i);
    cplx<T> a[12], b[12];
    load_stream<P>(x + h * k.hx, i, a);
    load_stream<P>(y + h * k.hy, i, b);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      re += (double)a[c].re * b[c].re + (double)a[c].im * b[c].im;
      im += (double)a[c].re * b[c].im - (double)a[c].im * b[c].re;
    }
  }
  double v[2] = {re, im};
  block_sum_store<2>(v, k.partials + (size_t)sys * 2 * k.nblk, k.nblk, blockIdx.x);
}

// ------------------------------------------------------------ finishing sums
constexpr int FIN_BS = 1024;

__global__ __launch_bounds__(FIN_BS) void k_finish_sums(const double *partials, unsigned nblocks, double *out,
                                                        int ostride, int accumulate, const int *skip, int sstride) {
  const int j = blockIdx.x;
  double v[1] = {0.0};
  for (unsigned b = threadIdx.x; b < nblocks; b += FIN_BS) v[0] += partials[(size_t)j * nblocks + b];
  block_sum_n<1>(v);
  if (threadIdx.x == 0 && !(skip && skip[(size_t)j * sstride])) {
    double *d = out + (size_t)j * ostride;
    *d = accumulate ? (*d + v[0]) : v[0];
  }
}

// ------------------------------------------------------------ elementwise
// out = c * x + y  (out may alias y)
template <int P>
__global__ __launch_bounds__(BLAS_BS) void k_caxpy(KBlas k) {
  using T = RealOf<P>;
  const int sys = blockIdx.y;
  const long n = (long)k.v.vh * k.v.nhalf;
  const cplx<T> c = {(T)k.c_re, (T)k.c_im};
  for (long f = (long)blockIdx.x * BLAS_BS + threadIdx.x; f < n; f += (long)k.nblk * BLAS_BS) {
    int h, i;
    site_of(k.v, f, h, i);
    cplx<T> a[12], b[12];
    // both operands are read once: streaming loads
    load_stream<P>(k.x + sys * k.sx + h * k.hx, i, a);
    load_stream<P>(k.y + sys * k.sy + h * k.hy, i, b);
#pragma unroll
    for (int q = 0; q < 12; ++q) cfma(b[q], c, a[q]);
    Spinor<P>::store(k.out + sys * k.so + h * k.ho, i, b);
  }
}

// out(PO) = s * x(PI); s = c_re, or c_re / sqrt(sc[sys].rnorm2) when sc != 0.
// Also zero-fills padding slots so every output slot is defined.
template <int PI, int PO>
__global__ __launch_bounds__(BLAS_BS) void k_convert(KBlas k) {
  using TI = RealOf<PI>;
  using TO = RealOf<PO>;
  const int sys = blockIdx.y;
  double s = k.c_re;
  if (k.sc) s = k.c_re / sqrt(k.sc[sys].rnorm2);
  const long n = (long)k.v.vpad * k.v.nhalf;
  for (long f = (long)blockIdx.x * BLAS_BS + threadIdx.x; f < n; f += (long)k.nblk * BLAS_BS) {
    const int h = (int)(f / k.v.vpad);
    const int i = (int)(f - (long)h * k.v.vpad);
    cplx<TO> b[12];
    if (i < k.v.vh) {
      cplx<TI> a[12];
      Spinor<PI>::load(k.x + sys * k.sx + h * k.hx, i, a);
      if constexpr (PO == WD_F64) {
#pragma unroll
        for (int q = 0; q < 12; ++q) b[q] = {(TO)(s * (double)a[q].re), (TO)(s * (double)a[q].im)};
      } else {
        const TO sf = (TO)s;
#pragma unroll
        for (int q = 0; q < 12; ++q) b[q] = {sf * (TO)a[q].re, sf * (TO)a[q].im};
      }
    } else {
#pragma unroll
      for (int q = 0; q < 12; ++q) b[q] = {(TO)0, (TO)0};
    }
    Spinor<PO>::store(k.out + sys * k.so + h * k.ho, i, b);
  }
}

// out(F64) += sqrt(sc[sys].rnorm2) * c_re * e(PE)   (defect-correction update)
template <int PE>
__global__ __launch_bounds__(BLAS_BS) void k_accum(KBlas k) {
  using TE = RealOf<PE>;
  const int sys = blockIdx.y;
  const double s = k.c_re * sqrt(k.sc[sys].rnorm2);
  const long n = (long)k.v.vh * k.v.nhalf;
  for (long f = (long)blockIdx.x * BLAS_BS + threadIdx.x; f < n; f += (long)k.nblk * BLAS_BS) {
    int h, i;
    site_of(k.v, f, h, i);
    cplx<TE> e[12];
    cplx<double> x[12];
    Spinor<PE>::load(k.x + sys * k.sx + h * k.hx, i, e);
    char *o = k.out + sys * k.so + h * k.ho;
    Spinor<WD_F64>::load(o, i, x);
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      x[q].re = fma(s, (double)e[q].re, x[q].re);
      x[q].im = fma(s, (double)e[q].im, x[q].im);
    }
    Spinor<WD_F64>::store(o, i, x);
  }
}

// ------------------------------------------------------------ CG recurrences
// alpha = rr[j] / qq;  X += alpha P;  S -= alpha Q;  ss = |S|^2.
// x = X (precision PX), y = P, out = S, out2 = Q (precision PV) -- Q is read only.
template <int PX, int PV>
__global__ __launch_bounds__(BLAS_BS) void k_cg_update(KBlas k) {
  using TV = RealOf<PV>;
  using TX = RealOf<PX>;
  const int sys = blockIdx.y;
  CgScalars *sc = k.sc + sys;
  if (sc->done) return;
  const double qq = sc->qq;
  if (!(qq > 0.0) || !(qq < 1e300) || !(sc->rr[k.j] < 1e300)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->done = 2;  // breakdown / non-finite
    return;
  }
  const double alpha = sc->rr[k.j] / qq;
  const long n = (long)k.v.vh * k.v.nhalf;
  double acc = 0.0;
  for (long f = (long)blockIdx.x * BLAS_BS + threadIdx.x; f < n; f += (long)k.nblk * BLAS_BS) {
    int h, i;
    site_of(k.v, f, h, i);
    cplx<TV> p[12], s[12], q[12];
    cplx<TX> x[12];
    char *X = (char *)k.x + sys * k.sx + h * k.hx;
    const char *Pp = k.y + sys * k.sy + h * k.hy;
    char *S = k.out + sys * k.so + h * k.ho;
    const char *Q = k.out2 + sys * k.so2 + h * k.ho2;
    Spinor<PV>::load(Pp, i, p);
    Spinor<PV>::load(Q, i, q);
    Spinor<PV>::load(S, i, s);
    Spinor<PX>::load(X, i, x);
    const TV a = (TV)alpha;
    const TX ax = (TX)alpha;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      x[c].re = fma(ax, (TX)p[c].re, x[c].re);
      x[c].im = fma(ax, (TX)p[c].im, x[c].im);
      s[c].re = fma(-a, q[c].re, s[c].re);
      s[c].im = fma(-a, q[c].im, s[c].im);
    }
    Spinor<PX>::store(X, i, x);
    Spinor<PV>::store(S, i, s);
    if constexpr (PV == WD_F64 || PV == WD_F32) {
#pragma unroll
      for (int c = 0; c < 12; ++c) acc += (double)s[c].re * s[c].re + (double)s[c].im * s[c].im;
    } else {  // norm of the stored (rounded) residual
      cplx<TV> r[12];
      Spinor<PV>::load(S, i, r);
#pragma unroll
      for (int c = 0; c < 12; ++c) acc += (double)r[c].re * r[c].re + (double)r[c].im * r[c].im;
    }
  }
  double v[1] = {acc};
  block_sum_store<1>(v, k.partials + (size_t)sys * k.nblk, k.nblk, blockIdx.x);
}

// Second stage of the CG update: ss = sum of the block partials (block
// order), iteration count and convergence flags.  Systems that were done, or
// broke down in the update, are left alone.
__global__ __launch_bounds__(FIN_BS) void k_cg_update_finish(const double *partials, unsigned nblk, CgScalars *scs) {
  CgScalars *sc = scs + blockIdx.x;
  if (sc->done) return;
  double v[1] = {0.0};
  for (unsigned b = threadIdx.x; b < nblk; b += FIN_BS) v[0] += partials[(size_t)blockIdx.x * nblk + b];
  block_sum_n<1>(v);
  if (threadIdx.x == 0) {
    sc->ss = v[0];
    sc->iters += 1;
    if (v[0] <= sc->stop2) sc->done = 1;
    else if (sc->iters >= sc->max_iters) sc->done = 3;
  }
}

// beta = rr[1-j] / rr[j];  P = R + beta P.   x = R, out = P.
template <int PV>
__global__ __launch_bounds__(BLAS_BS) void k_cg_pupdate(KBlas k) {
  using TV = RealOf<PV>;
  const int sys = blockIdx.y;
  const CgScalars *sc = k.sc + sys;
  if (sc->done) return;
  const double beta = sc->rr[1 - k.j] / sc->rr[k.j];
  const TV b = (TV)beta;
  const long n = (long)k.v.vh * k.v.nhalf;
  for (long f = (long)blockIdx.x * BLAS_BS + threadIdx.x; f < n; f += (long)k.nblk * BLAS_BS) {
    int h, i;
    site_of(k.v, f, h, i);
    cplx<TV> r[12], p[12];
    char *Pp = k.out + sys * k.so + h * k.ho;
    Spinor<PV>::load(k.x + sys * k.sx + h * k.hx, i, r);
    Spinor<PV>::load(Pp, i, p);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      p[c].re = fma(b, p[c].re, r[c].re);
      p[c].im = fma(b, p[c].im, r[c].im);
    }
    Spinor<PV>::store(Pp, i, p);
  }
}

// ------------------------------------------------------------ launchers
static unsigned blocks_for(long n) {
  long b = (n + BLAS_BS - 1) / BLAS_BS;
  if (b > BLAS_MAX_BLOCKS) b = BLAS_MAX_BLOCKS;
  if (b < 1) b = 1;
  return (unsigned)b;
}

static VecGeom vgeom(const Geom &g, int nhalf, wd_prec p) {
  return VecGeom{g.vh, g.vpad, nhalf, half_bytes(g, p)};
}

#define WD_DISPATCH_P(prec, KERNEL, grid, k, st)                                               \
  switch (prec) {                                                                             \
    case WD_F64: hipLaunchKernelGGL(KERNEL<WD_F64>, grid, dim3(BLAS_BS), 0, st, k); break;    \
    case WD_F32: hipLaunchKernelGGL(KERNEL<WD_F32>, grid, dim3(BLAS_BS), 0, st, k); break;    \
    case WD_F16: hipLaunchKernelGGL(KERNEL<WD_F16>, grid, dim3(BLAS_BS), 0, st, k); break;    \
    case WD_BF16: hipLaunchKernelGGL(KERNEL<WD_BF16>, grid, dim3(BLAS_BS), 0, st, k); break;  \
    default: return set_error(WD_ERR_PREC, "blas: unknown precision %d", (int)prec);          \
  }

wd_status blas_norm2(const Geom &g, wd_prec prec, const VecRef &x, int nsys, RedBuf red, double *result,
                     hipStream_t st) {
  KBlas k{};
  k.v = vgeom(g, x.nhalf, prec);
  k.nblk = blocks_for((long)g.vh * x.nhalf);
  k.x = (const char *)x.p; k.sx = x.sys_stride; k.hx = k.v.half_stride;
  k.partials = red.partials; k.result = result;
  dim3 grid(k.nblk, (unsigned)nsys);
  WD_DISPATCH_P(prec, k_norm2, grid, k, st);
  WD_TRY(hip_check(hipGetLastError(), "norm2 launch"));
  return launch_finish_sums(red.partials, k.nblk, nsys, result, 1, 0, nullptr, 1, st);
}

wd_status blas_cdot(const Geom &g, wd_prec prec, const VecRef &x, const VecRef &y, int nsys, RedBuf red,
                    double *result, hipStream_t st) {
  KBlas k{};
  k.v = vgeom(g, x.nhalf, prec);
  k.nblk = blocks_for((long)g.vh * x.nhalf);
  k.x = (const char *)x.p; k.sx = x.sys_stride; k.hx = k.v.half_stride;
  k.y = (const char *)y.p; k.sy = y.sys_stride; k.hy = k.v.half_stride;
  k.partials = red.partials; k.result = result;
  dim3 grid(k.nblk, (unsigned)nsys);
  WD_DISPATCH_P(prec, k_cdot, grid, k, st);
  WD_TRY(hip_check(hipGetLastError(), "cdot launch"));
  return launch_finish_sums(red.partials, k.nblk, 2 * nsys, result, 1, 0, nullptr, 1, st);
}

wd_status blas_caxpy(const Geom &g, wd_prec prec, double cre, double cim, const VecRef &x, const VecRef &y,
                     int nsys, hipStream_t st) {
  KBlas k{};
  k.v = vgeom(g, x.nhalf, prec);
  k.nblk = blocks_for((long)g.vh * x.nhalf);
  k.x = (const char *)x.p; k.sx = x.sys_stride; k.hx = k.v.half_stride;
  k.y = (const char *)y.p; k.sy = y.sys_stride; k.hy = k.v.half_stride;
  k.out = (char *)y.p; k.so = y.sys_stride; k.ho = k.v.half_stride;
  k.c_re = cre; k.c_im = cim;
  dim3 grid(k.nblk, (unsigned)nsys);
  WD_DISPATCH_P(prec, k_caxpy, grid, k, st);
  return hip_check(hipGetLastError(), "caxpy launch");
}

template <int PI>
static void launch_convert_out(wd_prec po, dim3 grid, const KBlas &k, hipStream_t st) {
  switch (po) {
    case WD_F64: hipLaunchKernelGGL((k_convert<PI, WD_F64>), grid, dim3(BLAS_BS), 0, st, k); break;
    case WD_F32: hipLaunchKernelGGL((k_convert<PI, WD_F32>), grid, dim3(BLAS_BS), 0, st, k); break;
    case WD_F16: hipLaunchKernelGGL((k_convert<PI, WD_F16>), grid, dim3(BLAS_BS), 0, st, k); break;
    case WD_BF16: hipLaunchKernelGGL((k_convert<PI, WD_BF16>), grid, dim3(BLAS_BS), 0, st, k); break;
  }
}

wd_status blas_convert(const Geom &g, wd_prec pi, const VecRef &x, wd_prec po, const VecRef &out, double scale,
                       CgScalars *sc_inv_sqrt_rnorm, int nsys, hipStream_t st) {
  if ((unsigned)pi > 3u || (unsigned)po > 3u) return set_error(WD_ERR_PREC, "convert: bad precision");
  KBlas k{};
  k.v = vgeom(g, x.nhalf, pi);
  k.nblk = blocks_for((long)g.vpad * x.nhalf);
  k.x = (const char *)x.p; k.sx = x.sys_stride; k.hx = half_bytes(g, pi);
  k.out = (char *)out.p; k.so = out.sys_stride; k.ho = half_bytes(g, po);
  k.c_re = scale;
  k.sc = sc_inv_sqrt_rnorm;
  dim3 grid(k.nblk, (unsigned)nsys);
  switch (pi) {
    case WD_F64: launch_convert_out<WD_F64>(po, grid, k, st); break;
    case WD_F32: launch_convert_out<WD_F32>(po, grid, k, st); break;
    case WD_F16: launch_convert_out<WD_F16>(po, grid, k, st); break;
    case WD_BF16: launch_convert_out<WD_BF16>(po, grid, k, st); break;
  }
  return hip_check(hipGetLastError(), "convert launch");
}

wd_status blas_accum(const Geom &g, wd_prec pe, const VecRef &e, const VecRef &x64, double scale, CgScalars *sc,
                     int nsys, hipStream_t st) {
  KBlas k{};
  k.v = vgeom(g, e.nhalf, pe);
  k.nblk = blocks_for((long)g.vh * e.nhalf);
  k.x = (const char *)e.p; k.sx = e.sys_stride; k.hx = half_bytes(g, pe);
  k.out = (char *)x64.p; k.so = x64.sys_stride; k.ho = half_bytes(g, WD_F64);
  k.c_re = scale;
  k.sc = sc;
  dim3 grid(k.nblk, (unsigned)nsys);
  WD_DISPATCH_P(pe, k_accum, grid, k, st);
  return hip_check(hipGetLastError(), "accum launch");
}

template <int PX>
static void launch_cgu(wd_prec pv, dim3 grid, const KBlas &k, hipStream_t st) {
  switch (pv) {
    case WD_F64: hipLaunchKernelGGL((k_cg_update<PX, WD_F64>), grid, dim3(BLAS_BS), 0, st, k); break;
    case WD_F32: hipLaunchKernelGGL((k_cg_update<PX, WD_F32>), grid, dim3(BLAS_BS), 0, st, k); break;
    case WD_F16: hipLaunchKernelGGL((k_cg_update<PX, WD_F16>), grid, dim3(BLAS_BS), 0, st, k); break;
    case WD_BF16: hipLaunchKernelGGL((k_cg_update<PX, WD_BF16>), grid, dim3(BLAS_BS), 0, st, k); break;
  }
}

wd_status blas_cg_update(const Geom &g, wd_prec px, const VecRef &x, wd_prec pv, const VecRef &p, const VecRef &s,
                         const VecRef &q, CgScalars *sc, int j, int nsys, RedBuf red, hipStream_t st) {
  if (!((px == WD_F64 && pv == WD_F64) || (px == WD_F32 && pv != WD_F64)))
    return set_error(WD_ERR_PREC, "cg_update: unsupported precision pair");
  KBlas k{};
  k.v = vgeom(g, p.nhalf, pv);
  k.nblk = blocks_for((long)g.vh * p.nhalf);
  k.x = (const char *)x.p; k.sx = x.sys_stride; k.hx = half_bytes(g, px);
  k.y = (const char *)p.p; k.sy = p.sys_stride; k.hy = half_bytes(g, pv);
  k.out = (char *)s.p; k.so = s.sys_stride; k.ho = half_bytes(g, pv);
  k.out2 = (char *)q.p; k.so2 = q.sys_stride; k.ho2 = half_bytes(g, pv);
  k.sc = sc; k.j = j;
  k.partials = red.partials;
  dim3 grid(k.nblk, (unsigned)nsys);
  if (px == WD_F64) launch_cgu<WD_F64>(pv, grid, k, st);
  else launch_cgu<WD_F32>(pv, grid, k, st);
  WD_TRY(hip_check(hipGetLastError(), "cg_update launch"));
  hipLaunchKernelGGL(k_cg_update_finish, dim3((unsigned)nsys), dim3(FIN_BS), 0, st, (const double *)k.partials, k.nblk,
                     sc);
  return hip_check(hipGetLastError(), "cg_update finish launch");
}

wd_status blas_cg_pupdate(const Geom &g, wd_prec pv, const VecRef &r, const VecRef &p, CgScalars *sc, int j,
                          int nsys, hipStream_t st) {
  KBlas k{};
  k.v = vgeom(g, p.nhalf, pv);
  k.nblk = blocks_for((long)g.vh * p.nhalf);
  k.x = (const char *)r.p; k.sx = r.sys_stride; k.hx = half_bytes(g, pv);
  k.out = (char *)p.p; k.so = p.sys_stride; k.ho = half_bytes(g, pv);
  k.sc = sc; k.j = j;
  dim3 grid(k.nblk, (unsigned)nsys);
  WD_DISPATCH_P(pv, k_cg_pupdate, grid, k, st);
  return hip_check(hipGetLastError(), "cg_pupdate launch");
}

wd_status launch_finish_sums(const double *partials, unsigned nblocks, int n, double *out, int ostride,
                             int accumulate, const int *skip, int sstride, hipStream_t st) {
  if (n < 1) return WD_OK;
  hipLaunchKernelGGL(k_finish_sums, dim3((unsigned)n), dim3(FIN_BS), 0, st, partials, nblocks, out, ostride,
                     accumulate, skip, sstride);
  return hip_check(hipGetLastError(), "finishing sums launch");
}

}  // namespace wd
