// Layout conversion: canonical complex128 arrays <-> checkerboarded
// structure-of-arrays fields, and the hop-link arrays with 12-real
// compression (rows 0 and 1 of each SU(3) matrix; Sec. 5 counts 18 reals per
// link, of which the third row is redundant for SU(3)).
#include "wd_device.h"

namespace wd {

template <int P>
using RealOf = typename Spinor<P>::real;

struct KPack {
  Geom g;
  const double *canon;  // [V][12] complex128 as interleaved doubles
  double *canon_out;
  char *field;
  const char *field_in;
  int parity0, nparity;  // parities handled: parity0 .. parity0+nparity-1
  size_t half_stride;    // bytes between the two halves of a full field
};

__device__ __forceinline__ size_t canon_index(const Geom &g, int i, int parity) {
  const int x1h = i % g.L1h;
  const int rest = i / g.L1h;
  const int x2 = rest % g.L[1];
  const int r2 = rest / g.L[1];
  const int x3 = r2 % g.L[2];
  const int x4 = r2 / g.L[2];
  const int x1 = 2 * x1h + ((parity + x2 + x3 + x4) & 1);
  return (size_t)x1 + (size_t)g.L[0] * rest;
}

// Chiral basis -> storage basis (and back: S is an involution):
// spins (0,1) <- (psi_u + psi_l) / sqrt 2, spins (2,3) <- (psi_u - psi_l) / sqrt 2,
// computed as (a + b) * r and (a - b) * r with r = 1/sqrt 2 rounded to double.
__device__ __forceinline__ void to_storage_basis(const double *src, double (&o)[12][2]) {
  const double r = 0.70710678118654752440;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const double a = src[2 * c + q], b = src[2 * (c + 6) + q];
      o[c][q] = (a + b) * r;
      o[c + 6][q] = (a - b) * r;
    }
  }
}

template <int P>
__global__ __launch_bounds__(256) void k_pack_spinor(KPack k) {
  using T = RealOf<P>;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int h = blockIdx.y;  // which of the handled parities
  if (i >= k.g.vpad) return;
  const int parity = k.parity0 + h;
  char *dst = k.field + (size_t)h * k.half_stride;
  cplx<T> s[12];
  if (i < k.g.vh) {
    const size_t idx = canon_index(k.g, i, parity);
    const double *src = k.canon + idx * 24;
    double b[12][2];
    to_storage_basis(src, b);
#pragma unroll
    for (int c = 0; c < 12; ++c) s[c] = {(T)b[c][0], (T)b[c][1]};
  } else {
#pragma unroll
    for (int c = 0; c < 12; ++c) s[c] = {(T)0, (T)0};
  }
  Spinor<P>::store(dst, i, s);
}

template <int P>
__global__ __launch_bounds__(256) void k_unpack_spinor(KPack k) {
  using T = RealOf<P>;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int h = blockIdx.y;
  if (i >= k.g.vh) return;
  const int parity = k.parity0 + h;
  const char *src = k.field_in + (size_t)h * k.half_stride;
  cplx<T> s[12];
  Spinor<P>::load(src, i, s);
  const size_t idx = canon_index(k.g, i, parity);
  double *dst = k.canon_out + idx * 24;
  double b[12][2];
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    b[c][0] = (double)s[c].re;
    b[c][1] = (double)s[c].im;
  }
  double o[12][2];
  to_storage_basis(&b[0][0], o);  // S is its own inverse
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    dst[2 * c] = o[c][0];
    dst[2 * c + 1] = o[c][1];
  }
}

// Hop links: for output parity p and hop d, the matrix applied to the
// projected neighbour -- U_{x,mu} (d = mu) or U^dag_{x-mu,mu} (d = 4 + mu) --
// is stored at the output site's checkerboard slot, rows 0 and 1 only.
struct KPackGauge {
  Geom g;
  const double *U;  // [V][4][3][3] complex128
  char *l64;
  char *l32;
  size_t par64, par32;  // bytes per parity
};

__global__ __launch_bounds__(256) void k_pack_gauge(KPackGauge k) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int p = blockIdx.y;
  if (i >= k.g.vpad) return;
  int x[4] = {0, 0, 0, 0};
  const bool real_site = i < k.g.vh;
  if (real_site) {
    const int x1h = i % k.g.L1h;
    const int rest = i / k.g.L1h;
    x[1] = rest % k.g.L[1];
    const int r2 = rest / k.g.L[1];
    x[2] = r2 % k.g.L[2];
    x[3] = r2 / k.g.L[2];
    x[0] = 2 * x1h + ((p + x[1] + x[2] + x[3]) & 1);
  }
  for (int d = 0; d < 8; ++d) {
    const int mu = d & 3;
    double m[2][3][2];  // rows 0,1 of the hop matrix, (re, im)
    if (!real_site) {
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) m[r][c][0] = m[r][c][1] = 0.0;
    } else {
      int y[4] = {x[0], x[1], x[2], x[3]};
      if (d >= 4) y[mu] = (x[mu] == 0) ? k.g.L[mu] - 1 : x[mu] - 1;
      const size_t idx = (size_t)y[0] + (size_t)k.g.L[0] * (y[1] + (size_t)k.g.L[1] * (y[2] + (size_t)k.g.L[2] * y[3]));
      const double *u = k.U + (idx * 4 + mu) * 18;  // [row][col][re,im]
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) {
          if (d < 4) {
            m[r][c][0] = u[(r * 3 + c) * 2];
            m[r][c][1] = u[(r * 3 + c) * 2 + 1];
          } else {  // (U^dag)_{rc} = conj(U_{cr})
            m[r][c][0] = u[(c * 3 + r) * 2];
            m[r][c][1] = -u[(c * 3 + r) * 2 + 1];
          }
        }
    }
    v2d *d64 = (v2d *)(k.l64 + (size_t)p * k.par64);
    v4f *d32 = (v4f *)(k.l32 + (size_t)p * k.par32);
    // element order: (row 0: c0 c1 c2, row 1: c0 c1 c2)
    double e[6][2];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 3; ++c) {
        e[r * 3 + c][0] = m[r][c][0];
        e[r * 3 + c][1] = m[r][c][1];
      }
    for (int q = 0; q < 6; ++q) d64[link_packet<6>(d, q, i)] = v2d{e[q][0], e[q][1]};
    for (int q = 0; q < 3; ++q)
      d32[link_packet<3>(d, q, i)] =
          v4f{(float)e[2 * q][0], (float)e[2 * q][1], (float)e[2 * q + 1][0], (float)e[2 * q + 1][1]};
  }
}

static void parity_range(int parity, int &p0, int &np) {
  if (parity == WD_FULL) { p0 = 0; np = 2; }
  else { p0 = parity; np = 1; }
}

wd_status launch_pack_spinor(const wd_gauge *g, const void *canon, void *field, int parity, wd_prec prec,
                             hipStream_t st) {
  KPack k{};
  k.g = g->geom;
  k.canon = (const double *)canon;
  k.field = (char *)field;
  parity_range(parity, k.parity0, k.nparity);
  k.half_stride = half_bytes(g->geom, prec);
  dim3 grid((unsigned)((g->geom.vpad + 255) / 256), (unsigned)k.nparity);
  switch (prec) {
    case WD_F64: hipLaunchKernelGGL(k_pack_spinor<WD_F64>, grid, dim3(256), 0, st, k); break;
    case WD_F32: hipLaunchKernelGGL(k_pack_spinor<WD_F32>, grid, dim3(256), 0, st, k); break;
    case WD_F16: hipLaunchKernelGGL(k_pack_spinor<WD_F16>, grid, dim3(256), 0, st, k); break;
    case WD_BF16: hipLaunchKernelGGL(k_pack_spinor<WD_BF16>, grid, dim3(256), 0, st, k); break;
    default: return set_error(WD_ERR_PREC, "pack: unknown precision %d", (int)prec);
  }
  return hip_check(hipGetLastError(), "pack launch");
}

wd_status launch_unpack_spinor(const wd_gauge *g, const void *field, void *canon, int parity, wd_prec prec,
                               hipStream_t st) {
  KPack k{};
  k.g = g->geom;
  k.canon_out = (double *)canon;
  k.field_in = (const char *)field;
  parity_range(parity, k.parity0, k.nparity);
  k.half_stride = half_bytes(g->geom, prec);
  dim3 grid((unsigned)((g->geom.vpad + 255) / 256), (unsigned)k.nparity);
  switch (prec) {
    case WD_F64: hipLaunchKernelGGL(k_unpack_spinor<WD_F64>, grid, dim3(256), 0, st, k); break;
    case WD_F32: hipLaunchKernelGGL(k_unpack_spinor<WD_F32>, grid, dim3(256), 0, st, k); break;
    case WD_F16: hipLaunchKernelGGL(k_unpack_spinor<WD_F16>, grid, dim3(256), 0, st, k); break;
    case WD_BF16: hipLaunchKernelGGL(k_unpack_spinor<WD_BF16>, grid, dim3(256), 0, st, k); break;
    default: return set_error(WD_ERR_PREC, "unpack: unknown precision %d", (int)prec);
  }
  return hip_check(hipGetLastError(), "unpack launch");
}

wd_status launch_pack_gauge(const wd_gauge *g, const void *canon_dev, hipStream_t st) {
  KPackGauge k{};
  k.g = g->geom;
  k.U = (const double *)canon_dev;
  k.l64 = (char *)g->links64;
  k.l32 = (char *)g->links32;
  k.par64 = link_parity_bytes(g->geom, true);
  k.par32 = link_parity_bytes(g->geom, false);
  dim3 grid((unsigned)((g->geom.vpad + 255) / 256), 2);
  hipLaunchKernelGGL(k_pack_gauge, grid, dim3(256), 0, st, k);
  return hip_check(hipGetLastError(), "pack_gauge launch");
}

}  // namespace wd
