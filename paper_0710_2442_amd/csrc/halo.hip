// Time-slab decomposition on one device: the part of a multi-GPU hop that
// one GPU runs.  A rank owns the time slices [t0, t0 + nt) of the lattice;
// its fields hold only those slices (a contiguous, chunk-aligned range of
// checkerboard sites), and the neighbour spinors of its two time faces
// arrive as projected half spinors in two face buffers (the paper's
// T_ext message: 6 complex numbers per face site).
//
// Because every hop link is stored with its output site (the backward link
// U^dag_{x-4,4} of a bottom-face site included), a rank needs no links from
// its neighbours: the faces carry spinors only.
//
// k_halo_pack copies the half spinors of a rank's bottom (or top) slice that
// the rank below (above) needs; k_dslash_slab is the single-parity hop of a
// rank's slab, reading the time neighbours of its top and bottom slices from
// the face buffers.  The arithmetic is that of the full-lattice hop in the
// same order, so a set of ranks reproduces it bit for bit.
#include "wd_hop.h"

namespace wd {

namespace {

// Face buffers: the 6 complex numbers of a half spinor in 16-byte packets
// (FP64: 6, FP32: 3), chunked by 64 sites like the fields.
template <int P>
struct Half;
template <>
struct Half<WD_F64> {
  static constexpr int NP = 6;
  __device__ static void load(const void *b, size_t j, cplx<double> (&h)[6]) {
    const v2d *p = (const v2d *)b + (j >> 6) * (NP * 64) + (j & 63);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      v2d v = p[64 * c];
      h[c] = {v.x, v.y};
    }
  }
  __device__ static void store(void *b, size_t j, const cplx<double> (&h)[6]) {
    v2d *p = (v2d *)b + (j >> 6) * (NP * 64) + (j & 63);
#pragma unroll
    for (int c = 0; c < 6; ++c) p[64 * c] = v2d{h[c].re, h[c].im};
  }
};
template <>
struct Half<WD_F32> {
  static constexpr int NP = 3;
  __device__ static void load(const void *b, size_t j, cplx<float> (&h)[6]) {
    const v4f *p = (const v4f *)b + (j >> 6) * (NP * 64) + (j & 63);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      v4f v = p[64 * k];
      h[2 * k] = {v.x, v.y};
      h[2 * k + 1] = {v.z, v.w};
    }
  }
  __device__ static void store(void *b, size_t j, const cplx<float> (&h)[6]) {
    v4f *p = (v4f *)b + (j >> 6) * (NP * 64) + (j & 63);
#pragma unroll
    for (int k = 0; k < 3; ++k) p[64 * k] = v4f{h[2 * k].re, h[2 * k].im, h[2 * k + 1].re, h[2 * k + 1].im};
  }
};

struct KSlab {
  Geom g;
  int t0, nt;           // owned slices
  const char *in;       // input parity, owned slices only (local index = global - t0 * s4)
  char *out;            // output parity, owned slices only
  const char *face_lo;  // half spinors of slice t0 - 1 (from the rank below)
  const char *face_hi;  // half spinors of slice t0 + nt (from the rank above)
  const char *links;    // hop links of the output parity (global handle)
  double a;
  int parity;
};

// The time hop from a half spinor that arrived in a face buffer: the MU = 3
// branch of hop_term_u with the load replaced.
template <int P, int S>
__device__ __forceinline__ void time_hop_from_half(cplx<RealOf<P>> (&acc)[12], cplx<RealOf<P>> (&h)[6],
                                                   const cplx<RealOf<P>> (&u)[6], RealOf<P> sign) {
  using T = RealOf<P>;
  const T f = (T)2 * sign;
#pragma unroll
  for (int c = 0; c < 6; ++c) h[c] = f * h[c];
  cplx<T> r2[3];
  rebuild_row2(u, r2);
  cplx<T> g[6];
  {
    cplx<T> v[3] = {h[0], h[1], h[2]};
    cplx<T> y[3];
    su3_mul(u, r2, v, y);
    g[0] = y[0]; g[1] = y[1]; g[2] = y[2];
  }
  {
    cplx<T> v[3] = {h[3], h[4], h[5]};
    cplx<T> y[3];
    su3_mul(u, r2, v, y);
    g[3] = y[0]; g[4] = y[1]; g[5] = y[2];
  }
  reconstruct_add<3, S>(acc, g);
}

// 64-site blocks: a rank's share is small (131,072 sites per parity at
// 32^3x8; a face 16,384 sites), and 64-site blocks spread it over every CU
// where 256-site blocks left most of them idle
constexpr int SLAB_BS = 64;

template <int P, bool DAG>
__global__ __launch_bounds__(SLAB_BS) void k_dslash_slab(KSlab k) {
  using T = RealOf<P>;
  const int vs = k.g.s4;  // sites of one parity per slice
  const int il = blockIdx.x * SLAB_BS + threadIdx.x;
  if (il >= k.nt * vs) return;
  const int base = k.t0 * vs;
  const int i = base + il;  // global checkerboard index
  const Coords c = coords_of(k.g, i, k.parity);
  int nb[8];
  neighbours(k.g, c, i, nb);
  const T one = (T)1;
  const T sf = (c.x4 == k.g.L[3] - 1) ? (T)k.g.tbc : one;
  const T sb = (c.x4 == 0) ? (T)k.g.tbc : one;
  constexpr int F = DAG ? -1 : 1;
  constexpr int B = -F;
  const int j = i - c.x4 * vs;  // index within the slice (same for the time neighbours)
  cplx<T> acc[12];
#pragma unroll
  for (int q = 0; q < 12; ++q) acc[q] = {(T)0, (T)0};
  cplx<T> u[6];
  Link<T>::load(k.links, 0, i, u);
  hop_term_u<P, 0, F>(acc, k.in, nb[0] - base, u, one);
  Link<T>::load(k.links, 1, i, u);
  hop_term_u<P, 1, F>(acc, k.in, nb[1] - base, u, one);
  Link<T>::load(k.links, 2, i, u);
  hop_term_u<P, 2, F>(acc, k.in, nb[2] - base, u, one);
  Link<T>::load(k.links, 3, i, u);
  if (c.x4 == k.t0 + k.nt - 1) {
    cplx<T> h[6];
    Half<P>::load(k.face_hi, j, h);
    time_hop_from_half<P, F>(acc, h, u, sf);
  } else {
    hop_term_u<P, 3, F>(acc, k.in, nb[3] - base, u, sf);
  }
  Link<T>::load(k.links, 4, i, u);
  hop_term_u<P, 0, B>(acc, k.in, nb[4] - base, u, one);
  Link<T>::load(k.links, 5, i, u);
  hop_term_u<P, 1, B>(acc, k.in, nb[5] - base, u, one);
  Link<T>::load(k.links, 6, i, u);
  hop_term_u<P, 2, B>(acc, k.in, nb[6] - base, u, one);
  Link<T>::load(k.links, 7, i, u);
  if (c.x4 == k.t0) {
    cplx<T> h[6];
    Half<P>::load(k.face_lo, j, h);
    time_hop_from_half<P, B>(acc, h, u, sb);
  } else {
    hop_term_u<P, 3, B>(acc, k.in, nb[7] - base, u, sb);
  }
  const T a = (T)k.a;
#pragma unroll
  for (int q = 0; q < 12; ++q) acc[q] = a * acc[q];
  Spinor<P>::store(k.out, il, acc);
}

// face[j] = the (LOWER) half of input site (slice ts, in-slice index j) of a
// rank's slab.
template <int P, bool LOWER>
__global__ __launch_bounds__(SLAB_BS) void k_halo_pack(const char *in, int local_slice, int vs, char *face) {
  using T = RealOf<P>;
  const int j = blockIdx.x * SLAB_BS + threadIdx.x;
  if (j >= vs) return;
  cplx<T> h[6];
  Spinor<P>::template load_half<LOWER>(in, (size_t)local_slice * vs + j, h);
  Half<P>::store(face, j, h);
}

}  // namespace

size_t halo_face_bytes(const Geom &g, wd_prec prec) {
  const size_t per = (prec == WD_F64) ? 96 : 48;
  return per * (size_t)g.s4;
}

wd_status launch_halo_pack(const wd_gauge *g, const void *in_slab, int nt, int face, int dagger, wd_prec prec,
                           void *face_buf, hipStream_t st) {
  const Geom &G = g->geom;
  // the bottom face feeds the rank below's forward time hop (1 + F gamma_4),
  // the top face the rank above's backward one; F = +1, or -1 for the dagger
  const bool lower = (face == 0) ? (dagger != 0) : (dagger == 0);
  const int ls = (face == 0) ? 0 : nt - 1;
  const dim3 grid((unsigned)((G.s4 + SLAB_BS - 1) / SLAB_BS));
#define WD_PK(PR)                                                                                        \
  if (lower)                                                                                             \
    hipLaunchKernelGGL((k_halo_pack<PR, true>), grid, dim3(SLAB_BS), 0, st, (const char *)in_slab, ls, G.s4, \
                       (char *)face_buf);                                                                \
  else                                                                                                   \
    hipLaunchKernelGGL((k_halo_pack<PR, false>), grid, dim3(SLAB_BS), 0, st, (const char *)in_slab, ls, G.s4, \
                       (char *)face_buf);
  if (prec == WD_F64) { WD_PK(WD_F64) } else { WD_PK(WD_F32) }
#undef WD_PK
  return hip_check(hipGetLastError(), "halo pack launch");
}

wd_status launch_dslash_slab(const wd_gauge *g, const void *in_slab, const void *face_lo, const void *face_hi,
                             void *out_slab, double a, int parity, int t0, int nt, int dagger, wd_prec prec,
                             hipStream_t st) {
  KSlab k{};
  k.g = g->geom;
  k.t0 = t0;
  k.nt = nt;
  k.in = (const char *)in_slab;
  k.out = (char *)out_slab;
  k.face_lo = (const char *)face_lo;
  k.face_hi = (const char *)face_hi;
  const bool f64 = prec == WD_F64;
  k.links = (const char *)(f64 ? g->links64 : g->links32) + (size_t)parity * link_parity_bytes(g->geom, f64);
  k.a = a;
  k.parity = parity;
  const dim3 grid((unsigned)(((size_t)nt * k.g.s4 + SLAB_BS - 1) / SLAB_BS));
#define WD_SL(PR)                                                                                        \
  if (dagger) hipLaunchKernelGGL((k_dslash_slab<PR, true>), grid, dim3(SLAB_BS), 0, st, k);             \
  else hipLaunchKernelGGL((k_dslash_slab<PR, false>), grid, dim3(SLAB_BS), 0, st, k);
  if (f64) { WD_SL(WD_F64) } else { WD_SL(WD_F32) }
#undef WD_SL
  return hip_check(hipGetLastError(), "slab hop launch");
}

}  // namespace wd
