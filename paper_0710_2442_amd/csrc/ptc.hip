// Gauge-covariant parallel-transport convolution (PTC) network: forward,
// backward (input and weight gradients), loss and Adam, on gfx950.
//
// A layer maps C_in spinor fields to C_out fields:
//   y_{c'}(x) = sum_c sum_h W^{(h)}_{c'c} (T_h psi_c)(x),
// h = 0 (T_0 = 1), h = 1..4: T_{+mu} psi(x) = U_{x,mu} psi(x+mu),
// h = 5..8: T_{-mu} psi(x) = U^dag_{x-mu,mu} psi(x-mu), with the time-boundary
// factor of Eq. 3.  W^{(h)}_{c'c} is a complex 4x4 spin matrix, so every
// layer commutes with gauge transformations.  T_h for h >= 1 is exactly the
// transport of the hop kernel: the same hop-link arrays (U_{x,mu} and
// U^dag_{x-mu,mu} stored at x) and the same neighbour indices, applied to the
// full 4-spinor instead of a projected half spinor.
//
// Network: 1 -> 2 -> 1 channels, weights FP32 ([layer][h][c'][c][4][4] complex,
// 288 + 288 = 576 complex numbers), activations stored in BF16 (or FP32),
// spin matrices given in the chiral basis and rotated into the fields' storage
// basis for the kernels (the optimiser works on the chiral-basis values),
// arithmetic and gradients in FP32, reductions over sites in FP64 in a
// fixed order.
//
// Backward: the input gradient of a layer is the same layer applied with the
// adjoint weights W'^{(hbar)}_{c c'} = (W^{(h)}_{c'c})^dag, hbar the adjoint hop
// (T_{+mu}^dag = T_{-mu}), so it is a gather with no atomics.  The weight
// gradient G^{(h)}_{c'c}[s',s] = sum_x sum_a g_{c'}(x)[s',a] conj((T_h psi_c)(x)[s,a])
// is summed over a wave's sites in FP64 (through LDS), then over the block's
// waves and the blocks in FP64, each in a fixed order.
#include <math.h>
#include <string.h>

#include <new>
#include <vector>

#include "wd_blas.h"
#include "wd_device.h"
#include "wd_ptc.h"
#include "wd_solver.h"

namespace wd {

template <int P>
using RealOf = typename Spinor<P>::real;

constexpr int PTC_BS = 256;
constexpr int PTC_NW = 1152;  // floats in all weights

struct KPtc {
  Geom g;
  const char *links32;  // float hop links, parity 0 then parity 1
  size_t link_par;      // bytes per parity of the link arrays
  const char *in;       // C_in full fields (channel-major)
  char *out;            // C_out full fields
  size_t in_chan;       // bytes per input channel (full field)
  size_t out_chan;
  size_t in_half, out_half;  // bytes per half field
  const float *W;       // this layer's weights [9][cout][cin][4][4] (re, im)
  // weight gradient
  const char *gy;       // C_out full fields, FP32 gradients
  size_t gy_chan, gy_half;
  double *partials;     // [nblocks][nparam floats]
  int accumulate;       // add to existing partials
};

// Coordinates and neighbours of checkerboard site i on parity p (same
// arithmetic as the hop kernel).
struct PtcSite {
  int nb[8];
  float sf, sb;
};

__device__ __forceinline__ PtcSite ptc_site(const Geom &g, int i, int p) {
  PtcSite s;
  const int x1h = i % g.L1h;
  const int rest = i / g.L1h;
  const int x2 = rest % g.L[1];
  const int r2 = rest / g.L[1];
  const int x3 = r2 % g.L[2];
  const int x4 = r2 / g.L[2];
  const int x1 = 2 * x1h + ((p + x2 + x3 + x4) & 1);
  const int xp1 = (x1 + 1 == g.L[0]) ? 0 : x1 + 1;
  const int xm1 = (x1 == 0) ? g.L[0] - 1 : x1 - 1;
  s.nb[0] = (xp1 >> 1) + g.L1h * rest;
  s.nb[4] = (xm1 >> 1) + g.L1h * rest;
  s.nb[1] = i + ((x2 == g.L[1] - 1) ? -(g.L[1] - 1) * g.s2 : g.s2);
  s.nb[5] = i + ((x2 == 0) ? (g.L[1] - 1) * g.s2 : -g.s2);
  s.nb[2] = i + ((x3 == g.L[2] - 1) ? -(g.L[2] - 1) * g.s3 : g.s3);
  s.nb[6] = i + ((x3 == 0) ? (g.L[2] - 1) * g.s3 : -g.s3);
  s.nb[3] = i + ((x4 == g.L[3] - 1) ? -(g.L[3] - 1) * g.s4 : g.s4);
  s.nb[7] = i + ((x4 == 0) ? (g.L[3] - 1) * g.s4 : -g.s4);
  s.sf = (x4 == g.L[3] - 1) ? g.tbc : 1.0f;
  s.sb = (x4 == 0) ? g.tbc : 1.0f;
  return s;
}

// a[d] without dynamic register indexing (a rolled loop would spill it)
__device__ __forceinline__ int pick8(const int (&a)[8], int d) {
  int r = a[0];
#pragma unroll
  for (int j = 1; j < 8; ++j) r = (d == j) ? a[j] : r;
  return r;
}

// v = T_h psi_c at site (p, i); psi channel base `chan` (full field).
template <int PIN>
__device__ __forceinline__ void transport(const KPtc &k, const PtcSite &s, int p, int i, int h, const char *chan,
                                          cplx<float> (&v)[12]) {
  if (h == 0) {
    cplx<RealOf<PIN>> t[12];
    Spinor<PIN>::load(chan + (size_t)p * k.in_half, i, t);
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = {(float)t[c].re, (float)t[c].im};
    return;
  }
  const int d = h - 1;
  cplx<RealOf<PIN>> t[12];
  Spinor<PIN>::load(chan + (size_t)(1 - p) * k.in_half, pick8(s.nb, d), t);
  cplx<float> u[6], r2[3];
  Link<float>::load(k.links32 + (size_t)p * k.link_par, d, i, u);
  rebuild_row2(u, r2);
  const float sg = (d == 3) ? s.sf : ((d == 7) ? s.sb : 1.0f);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp) {
    cplx<float> a[3] = {{(float)t[3 * sp].re, (float)t[3 * sp].im},
                        {(float)t[3 * sp + 1].re, (float)t[3 * sp + 1].im},
                        {(float)t[3 * sp + 2].re, (float)t[3 * sp + 2].im}};
    cplx<float> y[3];
    su3_mul(u, r2, a, y);
    v[3 * sp] = sg * y[0];
    v[3 * sp + 1] = sg * y[1];
    v[3 * sp + 2] = sg * y[2];
  }
}

// t = the raw input spinor that hop h reads at site (p, i): the site itself
// for h = 0, else its neighbour in direction h - 1 (other parity).
template <int PIN>
__device__ __forceinline__ void load_source(const KPtc &k, const PtcSite &s, int p, int i, int h, const char *chan,
                                            cplx<float> (&v)[12]) {
  cplx<RealOf<PIN>> t[12];
  if (h == 0) Spinor<PIN>::load(chan + (size_t)p * k.in_half, i, t);
  else Spinor<PIN>::load(chan + (size_t)(1 - p) * k.in_half, pick8(s.nb, h - 1), t);
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] = {(float)t[c].re, (float)t[c].im};
}

// acc += sg U m on every spin of m, U = the hop link of direction d at (p, i)
__device__ __forceinline__ void transport_add(const KPtc &k, const PtcSite &s, int p, int i, int d,
                                              const cplx<float> (&m)[12], cplx<float> (&acc)[12]) {
  cplx<float> u[6], r2[3];
  Link<float>::load(k.links32 + (size_t)p * k.link_par, d, i, u);
  rebuild_row2(u, r2);
  const float sg = (d == 3) ? s.sf : ((d == 7) ? s.sb : 1.0f);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp) {
    cplx<float> a[3] = {m[3 * sp], m[3 * sp + 1], m[3 * sp + 2]};
    cplx<float> y[3];
    su3_mul(u, r2, a, y);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      acc[3 * sp + c].re = fmaf(sg, y[c].re, acc[3 * sp + c].re);
      acc[3 * sp + c].im = fmaf(sg, y[c].im, acc[3 * sp + c].im);
    }
  }
}

// acc += W v  (W: 4x4 complex on spin, v: 4 spins x 3 colours)
__device__ __forceinline__ void spin_mat_acc(const float *W, const cplx<float> (&v)[12], cplx<float> (&acc)[12]) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const cplx<float> w = {W[2 * (4 * sp + t)], W[2 * (4 * sp + t) + 1]};
#pragma unroll
      for (int a = 0; a < 3; ++a) cfma(acc[3 * sp + a], w, v[3 * t + a]);
    }
  }
}

// INPAR = -1: the input lives on both parities.  INPAR = q: the input is zero
// off parity q, so a site of parity q takes only the h = 0 term and a site of
// the other parity only the hops (h >= 1); the zero terms are not read.
template <int PIN, int POUT, int CIN, int COUT, int INPAR = -1>
__global__ __launch_bounds__(PTC_BS) void k_ptc_layer(KPtc k) {
  const int p = blockIdx.y;
  const int i = blockIdx.x * PTC_BS + threadIdx.x;
  if (i >= k.g.vpad) return;
  cplx<RealOf<POUT>> o[12];
  if (i >= k.g.vh) {
#pragma unroll
    for (int c = 0; c < 12; ++c) o[c] = {0, 0};
#pragma unroll
    for (int co = 0; co < COUT; ++co) Spinor<POUT>::store(k.out + co * k.out_chan + (size_t)p * k.out_half, i, o);
    return;
  }
  const PtcSite s = ptc_site(k.g, i, p);
  cplx<float> acc[COUT][12];
#pragma unroll
  for (int co = 0; co < COUT; ++co)
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[co][c] = {0.f, 0.f};
  const int h0 = (INPAR >= 0 && p != INPAR) ? 1 : 0;
  const int h1 = (INPAR >= 0 && p == INPAR) ? 1 : 9;
  if constexpr (COUT == 1 && CIN > 1) {
    // more inputs than outputs: mix the spins first (W and the link commute:
    // one acts on spin, the other on colour), then transport once per hop
    for (int h = h0; h < h1; ++h) {
      cplx<float> m[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) m[c] = {0.f, 0.f};
#pragma unroll
      for (int ci = 0; ci < CIN; ++ci) {
        cplx<float> v[12];
        load_source<PIN>(k, s, p, i, h, k.in + ci * k.in_chan, v);
        spin_mat_acc(k.W + 32 * (h * CIN + ci), v, m);
      }
      if (h == 0) {
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[0][c] = acc[0][c] + m[c];
      } else {
        transport_add(k, s, p, i, h - 1, m, acc[0]);
      }
    }
  } else {
    for (int h = h0; h < h1; ++h) {
#pragma unroll
      for (int ci = 0; ci < CIN; ++ci) {
        cplx<float> v[12];
        transport<PIN>(k, s, p, i, h, k.in + ci * k.in_chan, v);
#pragma unroll
        for (int co = 0; co < COUT; ++co) spin_mat_acc(k.W + 32 * ((h * COUT + co) * CIN + ci), v, acc[co]);
      }
    }
  }
#pragma unroll
  for (int co = 0; co < COUT; ++co) {
#pragma unroll
    for (int c = 0; c < 12; ++c) o[c] = {(RealOf<POUT>)acc[co][c].re, (RealOf<POUT>)acc[co][c].im};
    Spinor<POUT>::store(k.out + co * k.out_chan + (size_t)p * k.out_half, i, o);
  }
}

// Weight gradient of one layer: partials[block][f] (+)= block sum of the
// per-site products; f indexes the layer's floats [h][c'][c][s'][s](re,im).
// The products of one (h, c', c) chunk (32 floats per site) go through LDS:
// each wave writes its 64 sites' rows, then lane f < 32 adds column f over
// the 64 sites in FP64 (site order), and the block adds its 4 waves in FP64.
template <int PIN, int CIN, int COUT>
__global__ __launch_bounds__(PTC_BS) void k_ptc_wgrad(KPtc k) {
  constexpr int NF = 9 * COUT * CIN * 32;
  constexpr int NW = PTC_BS / 64;
  __shared__ float tile[NW][64][33];  // one chunk's products per wave (row padded: no bank conflicts)
  __shared__ double wsum[NW][NF];     // the waves' site sums
  const int p = blockIdx.y;
  const int i = blockIdx.x * PTC_BS + threadIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const bool live = i < k.g.vh;
  PtcSite s;
  cplx<float> gy[COUT][12];
  if (live) {
    s = ptc_site(k.g, i, p);
#pragma unroll
    for (int co = 0; co < COUT; ++co)
      Spinor<WD_F32>::load(k.gy + co * k.gy_chan + (size_t)p * k.gy_half, i, gy[co]);
  }
#pragma unroll
  for (int h = 0; h < 9; ++h) {
#pragma unroll
    for (int ci = 0; ci < CIN; ++ci) {
      cplx<float> v[12];
      if (live) {
        transport<PIN>(k, s, p, i, h, k.in + ci * k.in_chan, v);
      } else {
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = {0.f, 0.f};
      }
#pragma unroll
      for (int co = 0; co < COUT; ++co) {
        float row[32];
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            cplx<float> acc = {0.f, 0.f};
            if (live) {
#pragma unroll
              for (int a = 0; a < 3; ++a) {
                // gy[s',a] * conj(v[s,a])
                const cplx<float> g = gy[co][3 * sp + a], x = v[3 * t + a];
                acc.re += g.re * x.re + g.im * x.im;
                acc.im += g.im * x.re - g.re * x.im;
              }
            }
            row[2 * (4 * sp + t)] = acc.re;
            row[2 * (4 * sp + t) + 1] = acc.im;
          }
        }
#pragma unroll
        for (int f = 0; f < 32; ++f) tile[w][lane][f] = row[f];
        __builtin_amdgcn_wave_barrier();  // a wave's LDS accesses complete in order
        if (lane < 32) {
          double t = 0.0;
#pragma unroll 4
          for (int q = 0; q < 64; ++q) t += (double)tile[w][q][lane];
          wsum[w][((h * COUT + co) * CIN + ci) * 32 + lane] = t;
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
  }
  __syncthreads();
  const size_t blk = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
  for (int f = threadIdx.x; f < NF; f += PTC_BS) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) t += wsum[q][f];
    double *dst = k.partials + blk * NF + f;
    *dst = k.accumulate ? (*dst + t) : t;
  }
}

// grad[f] = sum over blocks of partials[b][f], in block order.
__global__ __launch_bounds__(256) void k_ptc_reduce(const double *partials, int nblk, int nf, float *grad) {
  const int f = blockIdx.x * 256 + threadIdx.x;
  if (f >= nf) return;
  double t = 0.0;
  for (int b = 0; b < nblk; ++b) t += partials[(size_t)b * nf + f];
  grad[f] = (float)t;
}

// Adjoint weights for the input gradient of a layer (cout x cin):
// Wa[hbar][c][c'] = (W[h][c'][c])^dag.
__global__ void k_ptc_adjoint(const float *W, float *Wa, int cout, int cin) {
  const int n = threadIdx.x + blockIdx.x * blockDim.x;
  const int tot = 9 * cout * cin;
  if (n >= tot) return;
  const int h = n / (cout * cin), co = (n / cin) % cout, ci = n % cin;
  const int hb = (h == 0) ? 0 : (h <= 4 ? h + 4 : h - 4);
  const float *src = W + 32 * ((h * cout + co) * cin + ci);
  float *dst = Wa + 32 * ((hb * cin + ci) * cout + co);
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      dst[2 * (4 * a + b)] = src[2 * (4 * b + a)];
      dst[2 * (4 * a + b) + 1] = -src[2 * (4 * b + a) + 1];
    }
}

// out = S M S for n complex 4x4 spin matrices (chiral <-> storage basis;
// S = (1/sqrt 2) [[1, 1], [1, -1]] in 2x2 blocks is real, symmetric, S^2 = 1).
__global__ void k_ptc_rotate(const float *M, float *out, int n) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  const float r = 0.70710678118654752440f;
  float S[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) S[a][b] = ((a & 1) == (b & 1)) ? ((a >= 2 && b >= 2) ? -r : r) : 0.f;
  const float *src = M + 32 * m;
  float T[4][4][2];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      float re = 0.f, im = 0.f;
      for (int j = 0; j < 4; ++j) {
        re += src[2 * (4 * a + j)] * S[j][b];
        im += src[2 * (4 * a + j) + 1] * S[j][b];
      }
      T[a][b][0] = re;
      T[a][b][1] = im;
    }
  float *dst = out + 32 * m;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      float re = 0.f, im = 0.f;
      for (int i = 0; i < 4; ++i) {
        re += S[a][i] * T[i][b][0];
        im += S[a][i] * T[i][b][1];
      }
      dst[2 * (4 * a + b)] = re;
      dst[2 * (4 * a + b) + 1] = im;
    }
}

// Loss pieces: d = y - e (FP32 full fields); gy = scale * d; each block
// stores its FP64 partial sum of |d|^2, which the finishing kernel adds up in
// block order.
__global__ __launch_bounds__(256) void k_ptc_loss(const char *y, const char *e, char *gy, Geom g, float scale,
                                                  double *partials) {
  const int p = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const size_t hb = (size_t)96 * g.vpad;  // one FP32 half field
  double acc = 0.0;
  if (i < g.vpad) {
    cplx<float> a[12], b[12];
    if (i < g.vh) {
      Spinor<WD_F32>::load(y + p * hb, i, a);
      Spinor<WD_F32>::load(e + p * hb, i, b);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        a[c] = a[c] - b[c];
        acc += (double)a[c].re * a[c].re + (double)a[c].im * a[c].im;
        a[c] = scale * a[c];
      }
    } else {
#pragma unroll
      for (int c = 0; c < 12; ++c) a[c] = {0.f, 0.f};
    }
    Spinor<WD_F32>::store(gy + p * hb, i, a);
  }
  double v[1] = {acc};
  block_sum_store<1>(v, partials, gridDim.x * gridDim.y, blockIdx.y * gridDim.x + blockIdx.x);
}

// Adam on the 1152 real parameters (real and imaginary parts separately).
__global__ void k_adam(float *w, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const float gj = g[j];
  const float mj = b1 * m[j] + (1.f - b1) * gj;
  const float vj = b2 * v[j] + (1.f - b2) * gj * gj;
  m[j] = mj;
  v[j] = vj;
  w[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
}


// ------------------------------------------------- FP16-product inference
// The even-parity application inside the solver may take its products in
// FP16 with FP32 sums (v_dot2_f32_f16: two products and an FP32 add in one
// instruction, twice the rate of FP32 FMAs) on FP16 copies of the links and
// weights.  The network is linear, so the input is scaled to unit RMS before
// it is rounded to FP16 (a small residual would otherwise sink into FP16's
// subnormal range) and the output is scaled back.
typedef __fp16 hv2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ hv2 pkh(float a, float b) { return __builtin_amdgcn_cvt_pkrtz(a, b); }
__device__ __forceinline__ hv2 as_hv2(uint32_t u) { return __builtin_bit_cast(hv2, u); }

// v packed for products with a (re, im) pair w:
//   acc.re += w.re v.re - w.im v.im = dot(w, (v.re, -v.im))
//   acc.im += w.re v.im + w.im v.re = dot(w, (v.im, v.re))
struct HPk {
  hv2 a, b;
};
__device__ __forceinline__ HPk hpk(float re, float im) { return {pkh(re, -im), pkh(im, re)}; }
__device__ __forceinline__ void hmac(cplx<float> &acc, hv2 w, const HPk &v) {
  acc.re = __builtin_amdgcn_fdot2(w, v.a, acc.re, false);
  acc.im = __builtin_amdgcn_fdot2(w, v.b, acc.im, false);
}

struct KPtcH {
  Geom g;
  const uint2 *links16;  // per parity: [chunk of 64 sites][d][3 packets][64 lanes], 2 (re, im) FP16 pairs each
  size_t link16_par;     // uint2 per parity
  const char *in;        // layer 1: even half (BF16); layer 2: 2 full-field channels (BF16)
  char *out;
  size_t in_half, in_chan, out_half, out_chan;
  const uint32_t *W16;   // this layer's weights as (re, im) FP16 pairs, same order as the FP32 weights
  const double *norm2;   // |network input|^2
  double nreal;          // real components of the network input
};

// input scale: sqrt(nreal / |x|^2), so the scaled input has unit RMS
__device__ __forceinline__ float ptc_h_scale(const KPtcH &k) {
  const double n2 = *k.norm2;
  return (n2 > 0.0 && n2 < 1e300) ? (float)sqrt(k.nreal / n2) : 1.0f;
}

__device__ __forceinline__ size_t link16_at(int d, int q, int i) {
  return ((size_t)(i >> 6) * 24 + (size_t)(d * 3 + q)) * 64 + (size_t)(i & 63);
}

// y = sg U v on every spin
__device__ __forceinline__ void transport_h(const hv2 (&u)[9], const HPk (&v)[12], float sg, cplx<float> (&y)[12]) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cplx<float> acc = {0.f, 0.f};
#pragma unroll
      for (int b = 0; b < 3; ++b) hmac(acc, u[3 * a + b], v[3 * sp + b]);
      y[3 * sp + a] = {sg * acc.re, sg * acc.im};
    }
}

// acc += W v, W: a 4x4 spin matrix as 16 packed (re, im) pairs
__device__ __forceinline__ void spin_mat_h(const uint32_t *W, const HPk (&v)[12], cplx<float> (&acc)[12]) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const hv2 w = as_hv2(W[4 * sp + t]);
#pragma unroll
      for (int a = 0; a < 3; ++a) hmac(acc[3 * sp + a], w, v[3 * t + a]);
    }
}

__device__ __forceinline__ void load_h(const char *base, int i, float sc, HPk (&v)[12]) {
  cplx<float> x[12];
  Spinor<WD_BF16>::load(base, i, x);
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] = hpk(sc * x[c].re, sc * x[c].im);
}

// In both layers the neighbour spinor(s) and link of hop d + 1 are loaded
// (raw) before hop d is computed, so a wave keeps loads in flight while it
// computes (9% faster than loading at the top of each hop).
struct RawH {
  v4u q[3];  // a BF16 spinor's 3 packets
  uint2 l[3];  // an FP16 link's 3 packets
};
__device__ __forceinline__ void raw_h(const KPtcH &k, const char *base, int site, int p, int d, int i, RawH &r) {
  const v4u *b = (const v4u *)base + chunk_base<Spinor<WD_BF16>::CHUNK>(site);
#pragma unroll
  for (int q = 0; q < 3; ++q) r.q[q] = b[64 * q];
  const uint2 *lb = k.links16 + (size_t)p * k.link16_par;
#pragma unroll
  for (int q = 0; q < 3; ++q) r.l[q] = lb[link16_at(d, q, i)];
}
__device__ __forceinline__ void unpack_spinor_h(const v4u (&q)[3], float sc, HPk (&v)[12]) {
#pragma unroll
  for (int kq = 0; kq < 3; ++kq) {
    const uint32_t w[4] = {q[kq].x, q[kq].y, q[kq].z, q[kq].w};
#pragma unroll
    for (int j = 0; j < 4; ++j)
      v[4 * kq + j] = hpk(sc * bf16_to_f32((uint16_t)(w[j] & 0xffffu)), sc * bf16_to_f32((uint16_t)(w[j] >> 16)));
  }
}
// an FP16 hop link: rows 0-1 as stored, row 2 rebuilt in FP32 from them
// (u[3a + b] = M_ab)
__device__ __forceinline__ void unpack_link_h(const uint2 (&l)[3], hv2 (&u)[9]) {
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    u[2 * q] = as_hv2(l[q].x);
    u[2 * q + 1] = as_hv2(l[q].y);
  }
  cplx<float> f[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) f[j] = {(float)u[j].x, (float)u[j].y};
  cplx<float> r2[3];
  rebuild_row2(f, r2);
#pragma unroll
  for (int a = 0; a < 3; ++a) u[6 + a] = pkh(r2[a].re, r2[a].im);
}

// Layer 1 of [N (x_e, 0)]_e (1 -> 2 channels, both parities, BF16 out): an
// even site takes only W^(0) x, an odd site only the 8 hops from its even
// neighbours.
__global__ __launch_bounds__(PTC_BS) void k_ptc_h_l1(KPtcH k) {
  const int p = blockIdx.y;
  const int i = blockIdx.x * PTC_BS + threadIdx.x;
  if (i >= k.g.vpad) return;
  cplx<float> acc[2][12];
#pragma unroll
  for (int co = 0; co < 2; ++co)
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[co][c] = {0.f, 0.f};
  if (i < k.g.vh) {
    const float sc = ptc_h_scale(k);
    if (p == 0) {
      HPk v[12];
      load_h(k.in, i, sc, v);
#pragma unroll
      for (int co = 0; co < 2; ++co) spin_mat_h(k.W16 + 16 * co, v, acc[co]);
    } else {
      const PtcSite s = ptc_site(k.g, i, 1);
      RawH nx;
      raw_h(k, k.in, s.nb[0], 1, 0, i, nx);
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        const RawH cur = nx;
        if (d < 7) raw_h(k, k.in, s.nb[d + 1], 1, d + 1, i, nx);
        HPk v[12];
        unpack_spinor_h(cur.q, sc, v);
        hv2 u[9];
        unpack_link_h(cur.l, u);
        const float sg = (d == 3) ? s.sf : ((d == 7) ? s.sb : 1.0f);
        cplx<float> y[12];
        transport_h(u, v, sg, y);
        HPk yv[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) yv[c] = hpk(y[c].re, y[c].im);
#pragma unroll
        for (int co = 0; co < 2; ++co) spin_mat_h(k.W16 + 16 * ((d + 1) * 2 + co), yv, acc[co]);
      }
    }
  }
#pragma unroll
  for (int co = 0; co < 2; ++co) Spinor<WD_BF16>::store(k.out + co * k.out_chan + (size_t)p * k.out_half, i, acc[co]);
}

// Layer 2 (2 -> 1 channels, even sites only; spins mixed before the
// transport), output scaled back and stored in POUT.
template <int POUT>
__global__ __launch_bounds__(PTC_BS) void k_ptc_h_l2(KPtcH k) {
  const int i = blockIdx.x * PTC_BS + threadIdx.x;
  if (i >= k.g.vpad) return;
  cplx<float> acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = {0.f, 0.f};
  if (i < k.g.vh) {
    const PtcSite s = ptc_site(k.g, i, 0);
    RawH n0, n1;  // the two channels at the next neighbour (links in n0)
    raw_h(k, k.in + k.in_half, s.nb[0], 0, 0, i, n0);
    {
      const v4u *b = (const v4u *)(k.in + k.in_chan + k.in_half) + chunk_base<Spinor<WD_BF16>::CHUNK>(s.nb[0]);
#pragma unroll
      for (int q = 0; q < 3; ++q) n1.q[q] = b[64 * q];
    }
#pragma unroll
    for (int ci = 0; ci < 2; ++ci) {
      HPk v[12];
      load_h(k.in + ci * k.in_chan, i, 1.0f, v);
      spin_mat_h(k.W16 + 16 * ci, v, acc);
    }
#pragma unroll 1
    for (int d = 0; d < 8; ++d) {
      const RawH c0 = n0;
      const v4u c1[3] = {n1.q[0], n1.q[1], n1.q[2]};
      if (d < 7) {
        const int nb = pick8(s.nb, d + 1);
        raw_h(k, k.in + k.in_half, nb, 0, d + 1, i, n0);
        const v4u *b = (const v4u *)(k.in + k.in_chan + k.in_half) + chunk_base<Spinor<WD_BF16>::CHUNK>(nb);
#pragma unroll
        for (int q = 0; q < 3; ++q) n1.q[q] = b[64 * q];
      }
      cplx<float> m[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) m[c] = {0.f, 0.f};
      {
        HPk v[12];
        unpack_spinor_h(c0.q, 1.0f, v);
        spin_mat_h(k.W16 + 16 * ((d + 1) * 2), v, m);
        unpack_spinor_h(c1, 1.0f, v);
        spin_mat_h(k.W16 + 16 * ((d + 1) * 2 + 1), v, m);
      }
      HPk mv[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) mv[c] = hpk(m[c].re, m[c].im);
      hv2 u[9];
      unpack_link_h(c0.l, u);
      const float sg = (d == 3) ? s.sf : ((d == 7) ? s.sb : 1.0f);
      cplx<float> y[12];
      transport_h(u, mv, sg, y);
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[c] = acc[c] + y[c];
    }
    const float inv = 1.0f / ptc_h_scale(k);
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = {inv * acc[c].re, inv * acc[c].im};
  }
  cplx<RealOf<POUT>> o[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) o[c] = {(RealOf<POUT>)acc[c].re, (RealOf<POUT>)acc[c].im};
  Spinor<POUT>::store(k.out, i, o);
}

// FP16 copies: the hop links of both parities, and the weights
__global__ __launch_bounds__(256) void k_ptc_links16(const char *links32, size_t link_par, Geom g, uint2 *links16,
                                                      size_t link16_par) {
  const int p = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= g.vpad) return;
  for (int d = 0; d < 8; ++d) {
    cplx<float> u[6];
    if (i < g.vh) Link<float>::load<false>(links32 + (size_t)p * link_par, d, i, u);
    else
      for (int j = 0; j < 6; ++j) u[j] = {0.f, 0.f};
    for (int q = 0; q < 3; ++q) {
      const hv2 a = pkh(u[2 * q].re, u[2 * q].im), b = pkh(u[2 * q + 1].re, u[2 * q + 1].im);
      links16[(size_t)p * link16_par + link16_at(d, q, i)] =
          uint2{__builtin_bit_cast(uint32_t, a), __builtin_bit_cast(uint32_t, b)};
    }
  }
}

__global__ void k_ptc_w16(const float *W, uint32_t *W16, int n) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) W16[j] = __builtin_bit_cast(uint32_t, pkh(W[2 * j], W[2 * j + 1]));
}

// ------------------------------------------------- BF16 matrix-core inference
// [N (x_e, 0)]_e in two launches, BF16 operands, FP32 sums, BF16 hidden
// channels:
//   launch 1, odd sites o:  y_c(o) = sum_{h >= 1} W1^(h)_{c0} (T_h x)(o),  c = 0, 1
//   launch 2, even sites e: z(e) = Wc x(e) + sum_d s_d U_d(e) m_d(e),
//                           m_d(e) = sum_c W2^(d+1)_{0c} y_c(e + d)
// with Wc = sum_c W2^(0)_{0c} W1^(0)_{c0}: on the even sites layer 1 holds
// only W1^(0) x, which the h = 0 term of layer 2 multiplies by W2^(0), so the
// two spin matrices are multiplied once (per launch) instead of both being
// applied at every site.
//
// The spin mixing applies the same weights at every site: a contraction that
// runs on the matrix cores as v_mfma_f32_16x16x32_bf16 with 16 sites as the
// columns.  A wave takes 16 sites at a time; lane l serves site l % 16 and
// lane group g = l / 16 supplies the K values 8g .. 8g+7 of that site's
// column: the 4 spins (re, im) of one colour of one transported spinor (a
// direction in launch 1, a (direction, channel) pair in launch 2).  The 16
// rows of A are (channel or direction slot, spin, re/im) of the output; the
// weights enter A in real form, [[Wr, -Wi], [Wi, Wr]].  The transports (a
// different 3x3 matrix at every site) stay on the vector units as
// v_dot2_f32_bf16: two BF16 products added in FP32, with the spinor words
// used as stored (re, im) and the link entry in the forms (re, -im) and
// (im, re).  BF16 keeps FP32's exponent range, so no input scaling is needed.
//
// Lane layouts of v_mfma_f32_16x16x32_bf16 (wave64): A[m][k] in lane
// m + 16 (k / 8), element k % 8; B[k][n] in lane n + 16 (k / 8), element
// k % 8; D[m][n] in lane n + 16 (m / 4), element m % 4.
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t pk_bf(float re, float im) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f2v){re, im}, bf2v));
}
__device__ __forceinline__ float bdot(uint32_t a, uint32_t b, float c) {
  return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf2v, a), __builtin_bit_cast(bf2v, b), c, false);
}
// the same with the sum starting from zero: the three-operand encoding takes
// the constant, where the builtin's two-operand form needs a register zeroed
// first (one extra instruction per chain)
__device__ __forceinline__ float bdot0(uint32_t a, uint32_t b) {
  float r;
  asm("v_dot2_f32_bf16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ bf8v bf8_of(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  return __builtin_bit_cast(bf8v, v4u{a, b, c, d});
}
__device__ __forceinline__ f4v mfma_bf16(bf8v a, bf8v b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// q = n / d for n < 2^31 (umulhi(n, m) + n cannot overflow), with
// m = floor(2^32 (2^s - d) / d) + 1 and s = ceil(log2 d): the round-up
// multiplier of Granlund and Montgomery (PLDI 1994), exact for n < 2^32 / d * 2^s.
struct FDiv {
  uint32_t m;
  int s;
};
__device__ __forceinline__ int fdiv(int n, FDiv d) { return (int)((__umulhi((uint32_t)n, d.m) + (uint32_t)n) >> d.s); }

struct KPtcB {
  Geom g;
  FDiv dl1h, dl2, dl3;   // division by L1/2, L2, L3
  const uint2 *links;    // BF16 hop links, parity 0 then 1 (rows 0, 1 as (re, im) pairs; links16 layout)
  size_t link_par;       // uint2 per parity
  const char *x;         // BF16 even half (the network input)
  char *y;               // 2 BF16 odd half fields (hidden channels), colour-major: word 4a + s of a slot
  size_t y_chan;         // bytes per hidden channel
  char *out;             // even half, precision of launch 2's template argument
  const v4u *tabs;       // the A operands, per lane (see k_ptc_b_tables)
  int ngroups;           // groups of 16 sites: ceil(vh / 16)
};

// Coordinates of checkerboard site i on parity p, and its neighbours in
// direction mu (0..3, a per-lane value) forward (f) and backward (b), with the
// boundary factors of the time hops.
struct NbMu {
  int f, b;
  float sf, sb;
};
__device__ __forceinline__ NbMu nb_mu(const KPtcB &k, int i, int p, int mu) {
  const Geom &g = k.g;
  const int rest = fdiv(i, k.dl1h);
  const int x1h = i - rest * g.L1h;
  const int r2 = fdiv(rest, k.dl2);
  const int x2 = rest - r2 * g.L[1];
  const int x4 = fdiv(r2, k.dl3);
  const int x3 = r2 - x4 * g.L[2];
  NbMu n;
  // mu = 0
  const int x1 = 2 * x1h + ((p + x2 + x3 + x4) & 1);
  const int f0 = (((x1 + 1 == g.L[0]) ? 0 : x1 + 1) >> 1) + g.L1h * rest;
  const int b0 = (((x1 == 0) ? g.L[0] - 1 : x1 - 1) >> 1) + g.L1h * rest;
  // mu = 1..3: the coordinate, extent and stride of that direction
  const int x = (mu == 1) ? x2 : ((mu == 2) ? x3 : x4);
  const int L = (mu == 1) ? g.L[1] : ((mu == 2) ? g.L[2] : g.L[3]);
  const int s = (mu == 1) ? g.s2 : ((mu == 2) ? g.s3 : g.s4);
  const int fm = i + ((x == L - 1) ? -(L - 1) * s : s);
  const int bm = i + ((x == 0) ? (L - 1) * s : -s);
  n.f = (mu == 0) ? f0 : fm;
  n.b = (mu == 0) ? b0 : bm;
  n.sf = (mu == 3 && x4 == g.L[3] - 1) ? g.tbc : 1.0f;
  n.sb = (mu == 3 && x4 == 0) ? g.tbc : 1.0f;
  return n;
}

// The raw operands of one transport: a BF16 spinor (12 (re, im) words) and
// a BF16 link (rows 0, 1: 6 words).
struct RawB {
  v4u q[3];
  uint2 l[3];
};
// Loads at 32-bit byte offsets from a wave-uniform base (one address VGPR
// per load instead of a 64-bit add).
template <class T>
__device__ __forceinline__ T ld_at(const void *base, uint32_t off) {
  return *(const T *)((const char *)base + off);
}
// byte offset of packet q of BF16 spinor slot i
__device__ __forceinline__ uint32_t sp_off(int i, int q) {
  return (uint32_t)(((i >> 6) * Spinor<WD_BF16>::CHUNK + 64 * q + (i & 63)) * 16);
}
// byte offset of packet q of hop d's BF16 link at site i (links16 layout)
__device__ __forceinline__ uint32_t lk_off(int d, int q, int i) {
  return (uint32_t)((((i >> 6) * 24 + d * 3 + q) * 64 + (i & 63)) * 8);
}
__device__ __forceinline__ void load_spinor_b(const char *base, uint32_t chan_off, int site, v4u (&q)[3]) {
#pragma unroll
  for (int j = 0; j < 3; ++j) q[j] = ld_at<v4u>(base, chan_off + sp_off(site, j));
}
// links are read once per launch: streaming loads, so that they do not push
// the re-read spinors out of the L2
typedef uint32_t v2u __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void load_link_b(const uint2 *lb, int d, int i, uint2 (&l)[3]) {
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const v2u v = __builtin_nontemporal_load((const v2u *)((const char *)lb + lk_off(d, q, i)));
    l[q] = uint2{v.x, v.y};
  }
}
__device__ __forceinline__ uint32_t word_of(const v4u (&q)[3], int c) {
  const v4u v = q[c >> 2];
  return (c & 3) == 0 ? v.x : ((c & 3) == 1 ? v.y : ((c & 3) == 2 ? v.z : v.w));
}

// The 9 link entries M_ab in the two forms the dot products take:
// fr = (re, -im) gives Re(M_ab v_b), fi = (im, re) gives Im(M_ab v_b).  Row 2
// = conj(row0 x row1) is rebuilt from the forms of the BF16 rows with the
// same dot products (exact BF16 products, FP32 sums) and rounded to BF16:
//   row2_c = conj(a_p b_q - a_q b_p), (p, q) = (1, 2), (2, 0), (0, 1),
//   Re = Re(a_p b_q) - Re(a_q b_p),  -Im = Im(a_q b_p) - Im(a_p b_q),
// where -fr and -fi are the forms with both halves' signs flipped.  neg =
// 0x80008000 negates the whole link (a time-boundary factor of -1); it is
// nonzero only on the boundary slices, so the wave skips it elsewhere.
struct LinkB {
  uint32_t fr[9], fi[9];
};
__device__ __forceinline__ uint32_t rot16(uint32_t u) { return __builtin_amdgcn_alignbit(u, u, 16); }
__device__ __forceinline__ void link_forms(const uint2 (&l)[3], uint32_t neg, LinkB &L) {
  uint32_t u[6];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    u[2 * q] = l[q].x;
    u[2 * q + 1] = l[q].y;
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    L.fr[j] = u[j] ^ 0x80000000u;
    L.fi[j] = rot16(u[j]);
  }
  constexpr int P[3] = {1, 2, 0}, Q[3] = {2, 0, 1};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int p = P[c], q = Q[c];
    const float re = bdot(L.fr[p], u[3 + q], bdot0(L.fr[q] ^ 0x80008000u, u[3 + p]));
    const float im = bdot(L.fi[q], u[3 + p], bdot0(L.fi[p] ^ 0x80008000u, u[3 + q]));
    const uint32_t w = pk_bf(re, im);
    L.fr[6 + c] = w ^ 0x80000000u;
    L.fi[6 + c] = rot16(w);
  }
  if (__any(neg != 0u)) {
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      L.fr[j] ^= neg;
      L.fi[j] ^= neg;
    }
  }
}
// y = M v for one spin (v: its 3 colours as (re, im) words)
__device__ __forceinline__ void su3_b(const LinkB &L, uint32_t v0, uint32_t v1, uint32_t v2, cplx<float> (&y)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    y[a].re = bdot(L.fr[3 * a + 2], v2, bdot(L.fr[3 * a + 1], v1, bdot0(L.fr[3 * a], v0)));
    y[a].im = bdot(L.fi[3 * a + 2], v2, bdot(L.fi[3 * a + 1], v1, bdot0(L.fi[3 * a], v0)));
  }
}
// y += M v for one spin
__device__ __forceinline__ void su3_b_acc(const LinkB &L, uint32_t v0, uint32_t v1, uint32_t v2,
                                          cplx<float> (&y)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    y[a].re = bdot(L.fr[3 * a + 2], v2, bdot(L.fr[3 * a + 1], v1, bdot(L.fr[3 * a], v0, y[a].re)));
    y[a].im = bdot(L.fi[3 * a + 2], v2, bdot(L.fi[3 * a + 1], v1, bdot(L.fi[3 * a], v0, y[a].im)));
  }
}

// W in real form for A: row (.., s', rho), column (.., s, sigma) of the
// complex entry w = W_{s's}: rho = sigma -> Re w; (re, im) -> -Im w; (im, re) -> Im w
__device__ __forceinline__ float wreal(float wr, float wi, int rho, int sigma) {
  return (rho == sigma) ? wr : (rho == 0 ? -wi : wi);
}

// Groups of 16 sites per wave, in a grid-stride loop over the lattice in
// site order.  (Sweeps that give each XCD a box of the lattice, with grids
// of only the resident blocks, fetched more from beyond the L2, not less, and
// ran 3-5% slower.)
#define GROUP_SWEEP(k) \
  for (int grp = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6); grp < (k).ngroups; grp += (int)gridDim.x * 4)

// Padding lanes (site >= vh) compute on site vh - 1 and store nothing: a
// column of the matrix product depends only on its own site's data.
//
// Launch 1 (odd sites).  A: row m = 8c + 2s' + rho; K step j, lane group g:
// direction d = g + 4j (forward hops for j = 0, backward for j = 1).
__global__ __launch_bounds__(256) void k_ptc_b_l1(KPtcB k) {
  const int lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
  const bf8v A[2] = {__builtin_bit_cast(bf8v, k.tabs[lane]), __builtin_bit_cast(bf8v, k.tabs[64 + lane])};
  const uint2 *lb = k.links + k.link_par;  // odd-site links
  const int c_out = g >> 1, h_out = g & 1;
  const uint32_t y_off = (uint32_t)(c_out * k.y_chan);
  GROUP_SWEEP(k) {
    const int i0 = grp * 16 + col;
    const int i = min(i0, k.g.vh - 1);
    RawB r[2];
    const NbMu n = nb_mu(k, i, 1, g);
    load_spinor_b(k.x, 0, n.f, r[0].q);
    load_link_b(lb, g, i, r[0].l);
    load_spinor_b(k.x, 0, n.b, r[1].q);
    load_link_b(lb, g + 4, i, r[1].l);
    const uint32_t neg[2] = {n.sf < 0.f ? 0x80008000u : 0u, n.sb < 0.f ? 0x80008000u : 0u};
    f4v D[3];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      LinkB L;
      link_forms(r[j].l, neg[j], L);
      uint32_t bw[12];  // transported spinor, word 3s + a
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        cplx<float> y[3];
        su3_b(L, word_of(r[j].q, 3 * s), word_of(r[j].q, 3 * s + 1), word_of(r[j].q, 3 * s + 2), y);
#pragma unroll
        for (int a = 0; a < 3; ++a) bw[3 * s + a] = pk_bf(y[a].re, y[a].im);
      }
#pragma unroll
      for (int a = 0; a < 3; ++a)
        D[a] = mfma_bf16(A[j], bf8_of(bw[a], bw[3 + a], bw[6 + a], bw[9 + a]),
                         j == 0 ? (f4v){0.f, 0.f, 0.f, 0.f} : D[a]);
    }
    if (i0 < k.g.vh) {
      // rows 4g .. 4g+3: channel g / 2, spins 2h, 2h + 1 (h = g & 1), (re, im):
      // words 4a + 2h, 4a + 2h + 1 of the colour-major hidden channel
      char *yb = k.y + y_off;
#pragma unroll
      for (int a = 0; a < 3; ++a)
        *(uint2 *)(yb + sp_off(i, a) + 8 * h_out) = uint2{pk_bf(D[a][0], D[a][1]), pk_bf(D[a][2], D[a][3])};
    }
  }
}

// Launch 2 (even sites).  A (step j): row m = 8 slot + 2s' + rho, slot 0 ->
// direction j, slot 1 -> direction j + 4; lane group g supplies slot g / 2,
// channel g & 1, so A is zero where the row's slot is not the lane group's.
// D then holds m_d for lane group g's slot, spins 2 (g & 1) + t: each lane
// transports its two spins with U_d and keeps the sum over its slot's
// directions; lanes l and l ^ 32 (the two slots) add up at the end.  The
// Wc x(e) term is one more product with A nonzero only for slot 0 and lane
// group 0.
template <int POUT>
__global__ __launch_bounds__(256) void k_ptc_b_l2(KPtcB k) {
  const int lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
  bf8v A[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) A[j] = __builtin_bit_cast(bf8v, k.tabs[(2 + j) * 64 + lane]);
  const bf8v Ax = __builtin_bit_cast(bf8v, k.tabs[6 * 64 + lane]);
  const uint2 *lb = k.links;  // even-site links
  const int slot = g >> 1;
  const uint32_t y_off = (uint32_t)((g & 1) * k.y_chan);
  GROUP_SWEEP(k) {
    const int i0 = grp * 16 + col;
    const int i = min(i0, k.g.vh - 1);
    // slot 0: forward hops d = j, slot 1: backward hops d = j + 4, for mu = j
    int nb[4];
    uint32_t neg3 = 0u;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const NbMu n = nb_mu(k, i, 0, j);
      nb[j] = slot ? n.b : n.f;
      if (j == 3) neg3 = ((slot ? n.sb : n.sf) < 0.f) ? 0x80008000u : 0u;
    }
    // the Wc x(e) term first: it starts the sums (nonzero on lane groups 0, 1 only)
    cplx<float> acc[2][3];
    {
      v4u xq[3];
      load_spinor_b(k.x, 0, i, xq);
      f4v X[3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
        X[a] = mfma_bf16(Ax, bf8_of(word_of(xq, a), word_of(xq, 3 + a), word_of(xq, 6 + a), word_of(xq, 9 + a)),
                         (f4v){0.f, 0.f, 0.f, 0.f});
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[t][a] = {X[a][2 * t], X[a][2 * t + 1]};
    }
    // two steps in flight: step j + 2 is loaded once step j's operands are
    // used; the products of step j + 1 are started before step j's transports
    // (the matrix cores and the vector units work side by side)
    RawB cur[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      load_spinor_b(k.y, y_off, nb[j], cur[j].q);
      load_link_b(lb, j + 4 * slot, i, cur[j].l);
    }
    f4v M[3];  // the hidden channels are colour-major: packet a holds colour a's 4 spins
#pragma unroll
    for (int a = 0; a < 3; ++a) M[a] = mfma_bf16(A[0], __builtin_bit_cast(bf8v, cur[0].q[a]), (f4v){0.f, 0.f, 0.f, 0.f});
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      LinkB L;
      link_forms(cur[j & 1].l, 0u, L);
      f4v Mn[3];
      if (j < 3) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
          Mn[a] = mfma_bf16(A[j + 1], __builtin_bit_cast(bf8v, cur[(j + 1) & 1].q[a]), (f4v){0.f, 0.f, 0.f, 0.f});
      }
      if (j < 2) {
        load_spinor_b(k.y, y_off, nb[j + 2], cur[j].q);
        load_link_b(lb, j + 2 + 4 * slot, i, cur[j].l);
      }
      // the time-boundary factor of the x4 hops (step 3) on the mixed spinor
      const uint32_t ng = (j == 3) ? neg3 : 0u;
#pragma unroll
      for (int t = 0; t < 2; ++t)
        su3_b_acc(L, pk_bf(M[0][2 * t], M[0][2 * t + 1]) ^ ng, pk_bf(M[1][2 * t], M[1][2 * t + 1]) ^ ng,
                  pk_bf(M[2][2 * t], M[2][2 * t + 1]) ^ ng, acc[t]);
      if (j < 3) {
#pragma unroll
        for (int a = 0; a < 3; ++a) M[a] = Mn[a];
      }
    }
    // the two slots: lanes l (slot 0) and l + 32 (slot 1) hold the same spins
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        acc[t][a].re += __shfl_xor(acc[t][a].re, 32, 64);
        acc[t][a].im += __shfl_xor(acc[t][a].im, 32, 64);
      }
    if (i0 < k.g.vh && g < 2) {
      // components 6h .. 6h+5, h = g: (t, a) -> 3t + a
      const int h = g;
      if constexpr (POUT == WD_BF16) {
        uint32_t w[6];
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int a = 0; a < 3; ++a) w[3 * t + a] = pk_bf(acc[t][a].re, acc[t][a].im);
        if (h == 0) {
          *(v4u *)(k.out + sp_off(i, 0)) = v4u{w[0], w[1], w[2], w[3]};
          *(uint2 *)(k.out + sp_off(i, 1)) = uint2{w[4], w[5]};
        } else {
          *(uint2 *)(k.out + sp_off(i, 1) + 8) = uint2{w[0], w[1]};
          *(v4u *)(k.out + sp_off(i, 2)) = v4u{w[2], w[3], w[4], w[5]};
        }
      } else {
        v4f *p = (v4f *)k.out + chunk_base<Spinor<WD_F32>::CHUNK>(i) + 3 * 64 * h;
        const cplx<float> *z = &acc[0][0];
#pragma unroll
        for (int q = 0; q < 3; ++q) p[64 * q] = v4f{z[2 * q].re, z[2 * q].im, z[2 * q + 1].re, z[2 * q + 1].im};
      }
    }
  }
}

// The A operands of both launches for each of the 64 lanes, from the
// storage-basis weights W (both layers): T[j * 64 + lane], j = 0, 1: launch 1
// (K steps); 2..5: launch 2 (steps 0..3); 6: the Wc x(e) product.
constexpr int PTC_B_TABS = 7 * 64;  // v4u
__global__ __launch_bounds__(64) void k_ptc_b_tables(const float *W, v4u *T) {
  const int lane = threadIdx.x, g = lane >> 4, m = lane & 15;
  const int sp = (m >> 1) & 3, rho = m & 1;
  auto put = [&](int j, const float (&v)[8]) {
    T[j * 64 + lane] = v4u{pk_bf(v[0], v[1]), pk_bf(v[2], v[3]), pk_bf(v[4], v[5]), pk_bf(v[6], v[7])};
  };
  // launch 1: row m = 8c + 2s' + rho, K step j, lane group g: h = g + 4j + 1
  for (int j = 0; j < 2; ++j) {
    const int h = g + 4 * j + 1, c = m >> 3;
    float v[8];
    for (int e = 0; e < 8; ++e) {
      const float *w = W + 32 * (h * 2 + c) + 2 * (4 * sp + (e >> 1));
      v[e] = wreal(w[0], w[1], rho, e & 1);
    }
    put(j, v);
  }
  // launch 2: row m = 8 slot + 2s' + rho, lane group g: slot g / 2, channel g & 1
  const float *W2 = W + 576;
  const int slot_m = m >> 3;
  for (int j = 0; j < 4; ++j) {
    const int h = j + 4 * slot_m + 1, c = g & 1;
    float v[8];
    for (int e = 0; e < 8; ++e) {
      const float *w = W2 + 32 * (h * 2 + c) + 2 * (4 * sp + (e >> 1));
      v[e] = (slot_m == (g >> 1)) ? wreal(w[0], w[1], rho, e & 1) : 0.f;
    }
    put(2 + j, v);
  }
  // Wc[s'][s] = sum_c sum_t W2^(0)_{0c}[s'][t] W1^(0)_{c0}[t][s], slot 0 rows, lane group 0
  float v[8];
  for (int e = 0; e < 8; ++e) {
    const int s = e >> 1;
    cplx<float> wc = {0.f, 0.f};
    for (int c = 0; c < 2; ++c)
      for (int t = 0; t < 4; ++t) {
        const float *a = W2 + 32 * c + 2 * (4 * sp + t);
        const float *b = W + 32 * c + 2 * (4 * t + s);
        cfma(wc, cplx<float>{a[0], a[1]}, cplx<float>{b[0], b[1]});
      }
    v[e] = (slot_m == 0 && g == 0) ? wreal(wc.re, wc.im, rho, e & 1) : 0.f;
  }
  put(6, v);
}

// BF16 copy of the hop links of both parities (rows 0, 1; links16 layout)
__global__ __launch_bounds__(256) void k_ptc_links_bf16(const char *links32, size_t link_par, Geom g, uint2 *lb,
                                                         size_t lb_par) {
  const int p = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= g.vpad) return;
  for (int d = 0; d < 8; ++d) {
    cplx<float> u[6];
    if (i < g.vh) Link<float>::load<false>(links32 + (size_t)p * link_par, d, i, u);
    else
      for (int j = 0; j < 6; ++j) u[j] = {0.f, 0.f};
    for (int q = 0; q < 3; ++q)
      lb[(size_t)p * lb_par + link16_at(d, q, i)] =
          uint2{pk_bf(u[2 * q].re, u[2 * q].im), pk_bf(u[2 * q + 1].re, u[2 * q + 1].im)};
  }
}

}  // namespace wd

// ============================================================ host side
struct wd_ptc {
  const wd_gauge *g;
  float *Wc;       // device, the parameters: chiral-basis weights, 1152 floats
  float *gradc;    // device, gradient with respect to Wc
  float *W;        // device, the same weights in the storage spin basis (used by the kernels)
  float *Wadj;     // device, adjoint weights of both layers
  float *grad;     // device, 1152
  float *m, *v;    // Adam state
  int t;           // Adam steps taken
  wd_prec act;     // activation storage (WD_BF16 or WD_F32)
  void *x0, *y1, *y2, *gy2, *gy1;  // activations / gradients of one sample
  double *partials;                // wgrad partials: layer 1 then layer 2, nblk x 576 each
  double *scal;                    // [0] loss; [64..] reduction partials
  int nblk;                        // blocks of a full-lattice launch (both parities)
  // FP16-product inference (made on first use): FP16 hop links of both
  // parities, FP16 weights, and the input norm with its reduction partials
  uint2 *links16;
  uint32_t *W16;
  double *hnorm;
  // matrix-core inference: BF16 hop links of both parities (made on first
  // use) and the A operand tables (rebuilt whenever the weights change)
  uint2 *linksb;
  wd::v4u *tabs;
};

namespace wd {

static KPtc ptc_k(const wd_ptc *n) {
  KPtc k{};
  k.g = n->g->geom;
  k.links32 = (const char *)n->g->links32;
  k.link_par = link_parity_bytes(n->g->geom, false);
  return k;
}

static dim3 ptc_grid(const Geom &G) { return dim3((unsigned)((G.vpad + PTC_BS - 1) / PTC_BS), 2); }

template <int PIN, int POUT>
static void launch_layer(const KPtc &k, int cin, int cout, hipStream_t st) {
  const dim3 grid = ptc_grid(k.g);
  if (cin == 1 && cout == 2) hipLaunchKernelGGL((k_ptc_layer<PIN, POUT, 1, 2>), grid, dim3(PTC_BS), 0, st, k);
  else hipLaunchKernelGGL((k_ptc_layer<PIN, POUT, 2, 1>), grid, dim3(PTC_BS), 0, st, k);
}

static void dispatch_layer(const KPtc &k, wd_prec pin, wd_prec pout, int cin, int cout, hipStream_t st) {
  if (pin == WD_BF16 && pout == WD_BF16) launch_layer<WD_BF16, WD_BF16>(k, cin, cout, st);
  else if (pin == WD_BF16 && pout == WD_F32) launch_layer<WD_BF16, WD_F32>(k, cin, cout, st);
  else if (pin == WD_F32 && pout == WD_BF16) launch_layer<WD_F32, WD_BF16>(k, cin, cout, st);
  else launch_layer<WD_F32, WD_F32>(k, cin, cout, st);
}

// out (pout, cout channels) = layer(in (pin, cin channels)) with weights W.
static wd_status ptc_layer(const wd_ptc *n, const float *W, const void *in, wd_prec pin, int cin, void *out,
                           wd_prec pout, int cout, hipStream_t st) {
  KPtc k = ptc_k(n);
  k.in = (const char *)in;
  k.out = (char *)out;
  k.in_half = half_bytes(k.g, pin);
  k.out_half = half_bytes(k.g, pout);
  k.in_chan = 2 * k.in_half;
  k.out_chan = 2 * k.out_half;
  k.W = W;
  dispatch_layer(k, pin, pout, cin, cout, st);
  return hip_check(hipGetLastError(), "ptc layer");
}

// Weight-gradient partials of one layer (layer 0: 1 -> 2, layer 1: 2 -> 1).
static wd_status ptc_wgrad(const wd_ptc *n, int layer, const void *in, wd_prec pin, const void *gy, int accumulate,
                           hipStream_t st) {
  KPtc k = ptc_k(n);
  k.in = (const char *)in;
  k.in_half = half_bytes(k.g, pin);
  k.in_chan = 2 * k.in_half;
  k.gy = (const char *)gy;
  k.gy_half = half_bytes(k.g, WD_F32);
  k.gy_chan = 2 * k.gy_half;
  k.partials = n->partials + (size_t)layer * n->nblk * 576;
  k.accumulate = accumulate;
  const dim3 grid = ptc_grid(k.g);
#define WD_WG(PIN)                                                                                 \
  if (layer == 0) hipLaunchKernelGGL((k_ptc_wgrad<PIN, 1, 2>), grid, dim3(PTC_BS), 0, st, k); \
  else hipLaunchKernelGGL((k_ptc_wgrad<PIN, 2, 1>), grid, dim3(PTC_BS), 0, st, k);
  if (pin == WD_BF16) { WD_WG(WD_BF16) } else { WD_WG(WD_F32) }
#undef WD_WG
  return hip_check(hipGetLastError(), "ptc wgrad");
}

void ptc_release(wd_gauge *) {}

// Even-parity restriction of the network for the even-odd solver:
// out_e = [N (in_e, 0)]_e on half fields, input in pin and output in pout
// (FP32 or BF16).  The input's odd half is never read (layer 1 knows it is
// zero; with INPAR = 0 every read of the input lands in its even half, so a
// half field is a valid input) and layer 2 computes even sites only.  An
// input already in the activation precision is read in place.
template <int PA, int PO>
static void launch_even_l2(const KPtc &k, dim3 grid, hipStream_t st) {
  hipLaunchKernelGGL((k_ptc_layer<PA, PO, 2, 1>), grid, dim3(PTC_BS), 0, st, k);
}

wd_status ptc_apply_even(const wd_ptc *n, const void *in_even, wd_prec pin, void *out_even, wd_prec pout,
                         hipStream_t st) {
  const Geom &G = n->g->geom;
  if ((pin != WD_F32 && pin != WD_BF16) || (pout != WD_F32 && pout != WD_BF16))
    return set_error(WD_ERR_PREC, "ptc even: FP32 or BF16 fields");
  const void *x0 = in_even;
  if (pin != n->act) {
    WD_TRY(blas_convert(G, pin, vref(in_even, 1), n->act, vref(n->x0, 1), 1.0, nullptr, 1, st));
    x0 = n->x0;
  }
  KPtc k = ptc_k(n);
  k.in = (const char *)x0;
  k.out = (char *)n->y1;
  k.in_half = half_bytes(G, n->act);
  k.out_half = k.in_half;
  k.in_chan = 2 * k.in_half;
  k.out_chan = 2 * k.out_half;
  k.W = n->W;
  const dim3 grid = ptc_grid(G);
  if (n->act == WD_BF16) hipLaunchKernelGGL((k_ptc_layer<WD_BF16, WD_BF16, 1, 2, 0>), grid, dim3(PTC_BS), 0, st, k);
  else hipLaunchKernelGGL((k_ptc_layer<WD_F32, WD_F32, 1, 2, 0>), grid, dim3(PTC_BS), 0, st, k);
  WD_TRY(hip_check(hipGetLastError(), "ptc layer"));
  KPtc k2 = ptc_k(n);
  k2.in = (const char *)n->y1;
  k2.out = (char *)out_even;
  k2.in_half = half_bytes(G, n->act);
  k2.in_chan = 2 * k2.in_half;
  k2.out_half = half_bytes(G, pout);
  k2.out_chan = 2 * k2.out_half;
  k2.W = n->W + 576;
  const dim3 grid_e(grid.x, 1);  // parity 0 only
  if (n->act == WD_BF16) {
    if (pout == WD_BF16) launch_even_l2<WD_BF16, WD_BF16>(k2, grid_e, st);
    else launch_even_l2<WD_BF16, WD_F32>(k2, grid_e, st);
  } else {
    if (pout == WD_BF16) launch_even_l2<WD_F32, WD_BF16>(k2, grid_e, st);
    else launch_even_l2<WD_F32, WD_F32>(k2, grid_e, st);
  }
  return hip_check(hipGetLastError(), "ptc layer");
}

static size_t links16_per_parity(const Geom &G) { return (size_t)G.vpad / 64 * 24 * 64; }

// FP16 links (once per handle) and FP16 weights (every call: training may
// have changed the weights)
static wd_status ptc_h_prepare(wd_ptc *n, hipStream_t st) {
  const Geom &G = n->g->geom;
  if (!n->links16) {
    const size_t par = links16_per_parity(G);
    WD_HIP(hipMalloc(&n->links16, 2 * par * sizeof(uint2)));
    WD_HIP(hipMalloc(&n->W16, 576 * sizeof(uint32_t)));
    hipLaunchKernelGGL(k_ptc_links16, dim3((G.vpad + 255) / 256, 2), dim3(256), 0, st, (const char *)n->g->links32,
                       link_parity_bytes(G, false), G, n->links16, par);
    WD_TRY(hip_check(hipGetLastError(), "ptc fp16 links"));
  }
  hipLaunchKernelGGL(k_ptc_w16, dim3(3), dim3(192), 0, st, (const float *)n->W, n->W16, 576);
  return hip_check(hipGetLastError(), "ptc fp16 weights");
}

// [N (x_e, 0)]_e with FP16 products and FP32 sums: x_e a BF16 even half
// field, norm2 -> |x_e|^2 on the device (sets the input scale), output in
// pout (FP32 or BF16).  Needs BF16 activations.
wd_status ptc_apply_even_h(const wd_ptc *nc, const void *in_even, void *out_even, wd_prec pout, const double *norm2,
                           hipStream_t st) {
  wd_ptc *n = const_cast<wd_ptc *>(nc);  // the FP16 copies are caches of the handle's own data
  if (n->act != WD_BF16) return set_error(WD_ERR_PREC, "FP16-product network: BF16 activations only");
  if (pout != WD_F32 && pout != WD_BF16) return set_error(WD_ERR_PREC, "FP16-product network: FP32 or BF16 output");
  WD_TRY(ptc_h_prepare(n, st));
  const Geom &G = n->g->geom;
  KPtcH k{};
  k.g = G;
  k.links16 = n->links16;
  k.link16_par = links16_per_parity(G);
  k.in = (const char *)in_even;
  k.out = (char *)n->y1;
  k.out_half = half_bytes(G, WD_BF16);
  k.out_chan = 2 * k.out_half;
  k.W16 = n->W16;
  k.norm2 = norm2;
  k.nreal = 24.0 * (double)G.vh;
  const dim3 grid = ptc_grid(G);
  hipLaunchKernelGGL(k_ptc_h_l1, grid, dim3(PTC_BS), 0, st, k);
  WD_TRY(hip_check(hipGetLastError(), "ptc fp16 layer 1"));
  KPtcH k2 = k;
  k2.in = (const char *)n->y1;
  k2.in_half = half_bytes(G, WD_BF16);
  k2.in_chan = 2 * k2.in_half;
  k2.out = (char *)out_even;
  k2.out_half = half_bytes(G, pout);
  k2.out_chan = 2 * k2.out_half;
  k2.W16 = n->W16 + 288;
  const dim3 grid_e(grid.x, 1);
  if (pout == WD_BF16) hipLaunchKernelGGL(k_ptc_h_l2<WD_BF16>, grid_e, dim3(PTC_BS), 0, st, k2);
  else hipLaunchKernelGGL(k_ptc_h_l2<WD_F32>, grid_e, dim3(PTC_BS), 0, st, k2);
  return hip_check(hipGetLastError(), "ptc fp16 layer 2");
}

static FDiv make_fdiv(int d) {
  int s = 0;
  while ((1u << s) < (unsigned)d) ++s;
  const uint64_t m = (((uint64_t)1 << 32) * (((uint64_t)1 << s) - (uint64_t)d)) / (uint64_t)d + 1;
  return FDiv{(uint32_t)m, s};
}

// [N (x_e, 0)]_e on the matrix cores: x_e an even half field in pin (FP32
// input is first rounded to BF16 in the handle's x0 buffer), output in pout
// (FP32 or BF16).  Needs BF16 activations (the hidden channels are the
// handle's y1 buffer, odd halves only).
wd_status ptc_apply_even_b(const wd_ptc *nc, const void *in_even, wd_prec pin, void *out_even, wd_prec pout,
                           hipStream_t st) {
  wd_ptc *n = const_cast<wd_ptc *>(nc);  // the BF16 links are a cache of the handle's own data
  if (n->act != WD_BF16) return set_error(WD_ERR_PREC, "matrix-core network: BF16 activations only");
  if ((pin != WD_F32 && pin != WD_BF16) || (pout != WD_F32 && pout != WD_BF16))
    return set_error(WD_ERR_PREC, "matrix-core network: FP32 or BF16 fields");
  const Geom &G = n->g->geom;
  if ((size_t)G.vpad * 192 > 0xffffffffu)
    return set_error(WD_ERR_DIMS, "matrix-core network: %d sites per parity exceed its 32-bit offsets", G.vh);
  if (pin != WD_BF16) {
    WD_TRY(blas_convert(G, pin, vref(in_even, 1), WD_BF16, vref(n->x0, 1), 1.0, nullptr, 1, st));
    in_even = n->x0;
  }
  const size_t par = links16_per_parity(G);
  if (!n->linksb) {
    WD_HIP(hipMalloc(&n->linksb, 2 * par * sizeof(uint2)));
    hipLaunchKernelGGL(k_ptc_links_bf16, dim3((G.vpad + 255) / 256, 2), dim3(256), 0, st,
                       (const char *)n->g->links32, link_parity_bytes(G, false), G, n->linksb, par);
    WD_TRY(hip_check(hipGetLastError(), "ptc bf16 links"));
  }
  KPtcB k{};
  k.g = G;
  k.dl1h = make_fdiv(G.L1h);
  k.dl2 = make_fdiv(G.L[1]);
  k.dl3 = make_fdiv(G.L[2]);
  k.links = n->linksb;
  k.link_par = par;
  k.x = (const char *)in_even;
  k.y = (char *)n->y1;
  k.y_chan = half_bytes(G, WD_BF16);
  k.out = (char *)out_even;
  k.tabs = n->tabs;
  k.ngroups = (G.vh + 15) / 16;
  // 4 groups per block pass, at most 16 blocks per CU of 256 (the loop
  // strides over the rest)
  const unsigned nblk = (unsigned)std::max(1L, std::min<long>(((long)k.ngroups + 3) / 4, 256L * 16));
  hipLaunchKernelGGL(k_ptc_b_l1, dim3(nblk), dim3(256), 0, st, k);
  WD_TRY(hip_check(hipGetLastError(), "ptc matrix-core layer 1"));
  if (pout == WD_BF16) hipLaunchKernelGGL(k_ptc_b_l2<WD_BF16>, dim3(nblk), dim3(256), 0, st, k);
  else hipLaunchKernelGGL(k_ptc_b_l2<WD_F32>, dim3(nblk), dim3(256), 0, st, k);
  return hip_check(hipGetLastError(), "ptc matrix-core layer 2");
}

// N(in): F32 full field -> F32 full field; input and hidden layer are stored
// in the activation precision.
wd_status ptc_apply(const wd_ptc *n, const void *in, void *out, hipStream_t st) {
  const Geom &G = n->g->geom;
  WD_TRY(blas_convert(G, WD_F32, vref(in, 2), n->act, vref(n->x0, 2), 1.0, nullptr, 1, st));
  WD_TRY(ptc_layer(n, n->W, n->x0, n->act, 1, n->y1, n->act, 2, st));
  WD_TRY(ptc_layer(n, n->W + 576, n->y1, n->act, 2, out, WD_F32, 1, st));
  return WD_OK;
}

static wd_status ptc_alloc(wd_ptc *n) {
  const Geom &G = n->g->geom;
  const size_t fa = 2 * half_bytes(G, n->act), f32 = 2 * half_bytes(G, WD_F32);
  n->nblk = (int)((G.vpad + PTC_BS - 1) / PTC_BS) * 2;
  WD_HIP(hipMalloc(&n->W, PTC_NW * sizeof(float)));
  WD_HIP(hipMalloc(&n->Wc, PTC_NW * sizeof(float)));
  WD_HIP(hipMalloc(&n->gradc, PTC_NW * sizeof(float)));
  WD_HIP(hipMalloc(&n->Wadj, PTC_NW * sizeof(float)));
  WD_HIP(hipMalloc(&n->grad, PTC_NW * sizeof(float)));
  WD_HIP(hipMalloc(&n->m, PTC_NW * sizeof(float)));
  WD_HIP(hipMalloc(&n->v, PTC_NW * sizeof(float)));
  WD_HIP(hipMemset(n->m, 0, PTC_NW * sizeof(float)));
  WD_HIP(hipMemset(n->v, 0, PTC_NW * sizeof(float)));
  WD_HIP(hipMalloc(&n->x0, fa));
  WD_HIP(hipMalloc(&n->y1, 2 * fa));
  WD_HIP(hipMalloc(&n->y2, f32));
  WD_HIP(hipMalloc(&n->gy2, f32));
  WD_HIP(hipMalloc(&n->gy1, 2 * f32));
  WD_HIP(hipMalloc(&n->partials, (size_t)2 * n->nblk * 576 * sizeof(double)));
  WD_HIP(hipMalloc(&n->scal, (size_t)(n->nblk + 64) * sizeof(double)));
  WD_HIP(hipMalloc(&n->tabs, PTC_B_TABS * sizeof(v4u)));
  return WD_OK;
}

static void ptc_free(wd_ptc *n) {
  void *ps[] = {n->Wc,  n->gradc, n->W,  n->Wadj,     n->grad, n->m,   n->v,       n->x0,  n->y1,    n->y2,
                n->gy2, n->gy1,   n->partials, n->scal, n->links16, n->W16, n->hnorm, n->linksb, n->tabs};
  for (void *p : ps)
    if (p) (void)hipFree(p);
  delete n;
}

// Loss and gradients of a batch of B normalised pairs (r_b, e_b), F32 full
// fields, B of each, consecutive.  n->grad receives dL/dRe W + i dL/dIm W of
// L = (1/B) sum_b |N(r_b) - e_b|^2; n->scal[0] receives L * B.
static wd_status ptc_loss_grad(wd_ptc *n, const void *r, const void *e, int B, hipStream_t st) {
  const Geom &G = n->g->geom;
  const size_t f32 = 2 * half_bytes(G, WD_F32);
  WD_HIP(hipMemsetAsync(n->scal, 0, sizeof(double), st));
  hipLaunchKernelGGL(k_ptc_adjoint, dim3(1), dim3(64), 0, st, (const float *)n->W, n->Wadj, 2, 1);
  hipLaunchKernelGGL(k_ptc_adjoint, dim3(1), dim3(64), 0, st, (const float *)(n->W + 576), n->Wadj + 576, 1, 2);
  WD_HIP(hipGetLastError());
  for (int b = 0; b < B; ++b) {
    const char *rb = (const char *)r + (size_t)b * f32;
    const char *eb = (const char *)e + (size_t)b * f32;
    WD_TRY(blas_convert(G, WD_F32, vref(rb, 2), n->act, vref(n->x0, 2), 1.0, nullptr, 1, st));
    WD_TRY(ptc_layer(n, n->W, n->x0, n->act, 1, n->y1, n->act, 2, st));
    WD_TRY(ptc_layer(n, n->W + 576, n->y1, n->act, 2, n->y2, WD_F32, 1, st));
    hipLaunchKernelGGL(k_ptc_loss, ptc_grid(G), dim3(256), 0, st, (const char *)n->y2, eb, (char *)n->gy2, G,
                       2.0f / (float)B, n->scal + 64);
    WD_HIP(hipGetLastError());
    WD_TRY(launch_finish_sums(n->scal + 64, (unsigned)n->nblk, 1, n->scal, 1, 1, nullptr, 1, st));
    WD_TRY(ptc_wgrad(n, 1, n->y1, n->act, n->gy2, b > 0, st));
    // input gradient of layer 2 (adjoint weights: 1 -> 2 channels)
    WD_TRY(ptc_layer(n, n->Wadj + 576, n->gy2, WD_F32, 1, n->gy1, WD_F32, 2, st));
    WD_TRY(ptc_wgrad(n, 0, n->x0, n->act, n->gy1, b > 0, st));
  }
  hipLaunchKernelGGL(k_ptc_reduce, dim3((576 + 255) / 256), dim3(256), 0, st, (const double *)n->partials, n->nblk,
                     576, n->grad);
  hipLaunchKernelGGL(k_ptc_reduce, dim3((576 + 255) / 256), dim3(256), 0, st,
                     (const double *)(n->partials + (size_t)n->nblk * 576), n->nblk, 576, n->grad + 576);
  // gradient with respect to the chiral-basis parameters (W = S Wc S, S orthogonal and symmetric)
  hipLaunchKernelGGL(k_ptc_rotate, dim3(1), dim3(128), 0, st, (const float *)n->grad, n->gradc, PTC_NW / 32);
  return hip_check(hipGetLastError(), "ptc loss/grad");
}

// kernels' weights <- parameters (rotate every 4x4 block into the storage basis)
static wd_status ptc_sync_weights(wd_ptc *n, hipStream_t st) {
  hipLaunchKernelGGL(k_ptc_rotate, dim3(1), dim3(128), 0, st, (const float *)n->Wc, n->W, PTC_NW / 32);
  hipLaunchKernelGGL(k_ptc_b_tables, dim3(1), dim3(64), 0, st, (const float *)n->W, n->tabs);
  return hip_check(hipGetLastError(), "ptc rotate");
}

static wd_status check_pair_args(const wd_ptc *n, const void *r, const void *e, int B) {
  if (!n) return set_error(WD_ERR_ARG, "ptc handle is NULL");
  if (!r || !e) return set_error(WD_ERR_ARG, "ptc: NULL field pointer");
  if (B < 1 || B > 4096) return set_error(WD_ERR_ARG, "ptc: batch size %d", B);
  return hip_check(hipSetDevice(n->g->device), "hipSetDevice");
}

}  // namespace wd

using namespace wd;

extern "C" {

wd_status wd_ptc_create(const wd_gauge *g, const float *W_host, wd_prec act_prec, wd_ptc **out) {
  if (!out) return set_error(WD_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!g || !W_host) return set_error(WD_ERR_ARG, "ptc_create: NULL argument");
  if (act_prec != WD_F32 && act_prec != WD_BF16) return set_error(WD_ERR_PREC, "ptc activations: FP32 or BF16");
  for (int j = 0; j < PTC_NW; ++j)
    if (!isfinite(W_host[j])) return set_error(WD_ERR_NONFINITE, "ptc_create: weight %d is not finite", j);
  WD_HIP(hipSetDevice(g->device));
  wd_ptc *n = new (std::nothrow) wd_ptc();
  if (!n) return set_error(WD_ERR_OOM, "host allocation failed");
  memset(n, 0, sizeof(*n));
  n->g = g;
  n->act = act_prec;
  wd_status rc = ptc_alloc(n);
  if (rc == WD_OK) rc = hip_check(hipMemcpy(n->Wc, W_host, PTC_NW * sizeof(float), hipMemcpyHostToDevice), "weights");
  if (rc == WD_OK) rc = ptc_sync_weights(n, g->stream);
  if (rc == WD_OK) rc = hip_check(hipStreamSynchronize(g->stream), "weights");
  if (rc != WD_OK) {
    ptc_free(n);
    return rc;
  }
  *out = n;
  return WD_OK;
}

wd_status wd_ptc_destroy(wd_ptc *n) {
  if (!n) return WD_OK;
  (void)hipSetDevice(n->g->device);
  (void)hipDeviceSynchronize();
  ptc_free(n);
  return WD_OK;
}

wd_status wd_ptc_set_weights(wd_ptc *n, const float *W_host) {
  if (!n || !W_host) return set_error(WD_ERR_ARG, "NULL argument");
  WD_HIP(hipSetDevice(n->g->device));
  WD_HIP(hipStreamSynchronize(n->g->stream));
  WD_HIP(hipMemcpy(n->Wc, W_host, PTC_NW * sizeof(float), hipMemcpyHostToDevice));
  WD_TRY(ptc_sync_weights(n, n->g->stream));
  WD_HIP(hipStreamSynchronize(n->g->stream));
  WD_HIP(hipMemset(n->m, 0, PTC_NW * sizeof(float)));
  WD_HIP(hipMemset(n->v, 0, PTC_NW * sizeof(float)));
  n->t = 0;
  return WD_OK;
}

wd_status wd_ptc_get_weights(const wd_ptc *n, float *W_host) {
  if (!n || !W_host) return set_error(WD_ERR_ARG, "NULL argument");
  WD_HIP(hipSetDevice(n->g->device));
  WD_HIP(hipStreamSynchronize(n->g->stream));
  WD_HIP(hipMemcpy(W_host, n->Wc, PTC_NW * sizeof(float), hipMemcpyDeviceToHost));
  return WD_OK;
}

wd_status wd_ptc_apply(const wd_ptc *n, const void *in, void *out) {
  if (!n || !in || !out) return set_error(WD_ERR_ARG, "NULL argument");
  if (in == out) return set_error(WD_ERR_ARG, "ptc_apply: in and out must differ");
  WD_HIP(hipSetDevice(n->g->device));
  return ptc_apply(n, in, out, n->g->stream);
}

wd_status wd_ptc_apply_even(const wd_ptc *n, const void *in_even, wd_prec pin, void *out_even, wd_prec pout,
                            int flags) {
  if (!n || !in_even || !out_even) return set_error(WD_ERR_ARG, "NULL argument");
  if (in_even == out_even) return set_error(WD_ERR_ARG, "ptc_apply_even: in and out must differ");
  if ((flags & ~(WD_PTC_FP16_PRODUCTS | WD_PTC_BF16_MFMA)) || flags == (WD_PTC_FP16_PRODUCTS | WD_PTC_BF16_MFMA))
    return set_error(WD_ERR_ARG, "ptc_apply_even: unknown flags 0x%x", flags);
  if ((pin != WD_F32 && pin != WD_BF16) || (pout != WD_F32 && pout != WD_BF16))
    return set_error(WD_ERR_PREC, "ptc_apply_even: FP32 or BF16 fields");
  if (flags && n->act != WD_BF16)
    return set_error(WD_ERR_PREC, "ptc_apply_even: FP16 or BF16 products need BF16 activations");
  WD_HIP(hipSetDevice(n->g->device));
  hipStream_t st = n->g->stream;
  if (!flags) return ptc_apply_even(n, in_even, pin, out_even, pout, st);
  wd_ptc *m = const_cast<wd_ptc *>(n);
  const Geom &G = n->g->geom;
  if (flags & WD_PTC_BF16_MFMA) return ptc_apply_even_b(n, in_even, pin, out_even, pout, st);
  if (!m->hnorm) {
    WD_HIP(hipMalloc(&m->hnorm, (64 + 2 * (size_t)BLAS_MAX_BLOCKS) * sizeof(double)));
  }
  const void *x = in_even;
  if (pin != WD_BF16) {
    WD_TRY(blas_convert(G, pin, vref(in_even, 1), WD_BF16, vref(m->x0, 1), 1.0, nullptr, 1, st));
    x = m->x0;
  }
  WD_TRY(blas_norm2(G, WD_BF16, vref(x, 1), 1, RedBuf{m->hnorm + 64}, m->hnorm, st));
  return ptc_apply_even_h(n, x, out_even, pout, m->hnorm, st);
}

wd_status wd_ptc_loss_grad(wd_ptc *n, const void *r, const void *e, int B, double *loss, float *grad_host) {
  WD_TRY(check_pair_args(n, r, e, B));
  hipStream_t st = n->g->stream;
  WD_TRY(ptc_loss_grad(n, r, e, B, st));
  double l = 0;
  WD_HIP(hipMemcpyAsync(&l, n->scal, sizeof(double), hipMemcpyDeviceToHost, st));
  if (grad_host) WD_HIP(hipMemcpyAsync(grad_host, n->gradc, PTC_NW * sizeof(float), hipMemcpyDeviceToHost, st));
  WD_HIP(hipStreamSynchronize(st));
  if (loss) *loss = l / B;
  return WD_OK;
}

wd_status wd_ptc_train_step(wd_ptc *n, const void *r, const void *e, int B, double lr, double *loss) {
  WD_TRY(check_pair_args(n, r, e, B));
  if (!(lr > 0.0) || !isfinite(lr)) return set_error(WD_ERR_ARG, "ptc_train_step: lr must be > 0");
  hipStream_t st = n->g->stream;
  WD_TRY(ptc_loss_grad(n, r, e, B, st));
  n->t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)n->t), c2 = 1.f - powf(b2, (float)n->t);
  hipLaunchKernelGGL(k_adam, dim3((PTC_NW + 255) / 256), dim3(256), 0, st, n->Wc, (const float *)n->gradc, n->m,
                     n->v, PTC_NW, (float)lr, b1, b2, 1e-8f, c1, c2);
  WD_HIP(hipGetLastError());
  WD_TRY(ptc_sync_weights(n, st));
  if (loss) {
    double l = 0;
    WD_HIP(hipMemcpyAsync(&l, n->scal, sizeof(double), hipMemcpyDeviceToHost, st));
    WD_HIP(hipStreamSynchronize(st));
    *loss = l / B;
  }
  return WD_OK;
}

}  // extern "C"

namespace wd {
const wd_gauge *ptc_gauge(const wd_ptc *n) { return n->g; }
wd_prec ptc_act(const wd_ptc *n) { return n->act; }
}  // namespace wd
