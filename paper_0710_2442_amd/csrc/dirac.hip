// Full-lattice Wilson-Dirac operator (Eq. 3 on both checkerboards) in one
// launch, marching along x4 the way the paper streams a lattice that lives
// in main memory through on-chip storage a time slice at a time (Sec. 5).
//
// Every site's forward links serve two hops: U_{x,mu} for the forward hop of
// x and U^dag_{x,mu} for the backward hop of x + mu.  So do the spinors: a
// spinor psi_y is read by y's eight neighbours and, as X = psi for D_W, by
// y itself.  A lane owns one spatial site (x1, x2, x3) and walks a range of
// time slices; a block owns a tile of 256 spatial sites (a brick of whole x1
// rows, n2 rows deep in x2 and 2 planes in x3, where that fits the lattice,
// else 256 consecutive sites) and the same range.  At step k the lane
//   1. loads its own spinor psi(x, k), whose half kept by the forward time
//      projector finishes out(x, k-1) with the link U_{(x,k-1),4} carried from
//      the step before (then out(x, k-1) is stored);
//   2. loads its own time link U_{(x,k),4} and forms, from the other half of
//      psi(x, k), the backward time hop that out(x, k+1) receives (carried);
//   3. adds to that carried term the six spatial hops of (x, k): its own
//      spatial links, the neighbours' forward links as U^dag, and the
//      neighbours' spinors of slice k, all read in the same step by the
//      lanes that own them, so every byte of slice k is fetched from HBM
//      once and re-read within the step (from LDS in the staged form below,
//      else from L1 or L2); each direction's forward and backward hop run
//      back to back, so a spatial link's two reads are close together;
//   the partial output starts from the epilogue terms X - Y (taken before
//   the hops, so the own spinor is dead early) and every hop adds a times
//   its term.
// Across steps only three small objects move, in registers: the partial
// output (12 complex), the time link (6 complex) and the backward time term
// (6 complex).  The time neighbours, a whole slice of traffic apart in
// memory order, are therefore never fetched twice.  A range boundary costs
// one extra time link and half spinor on each side (per lane and range).
//
// Per site the launch moves 4 x 12 link reals + 24 input reals + 24 output
// reals (96 reals: 768 B in FP64), against 2 x 144 reals for two
// single-parity launches.
//
// Blocks go round robin to the 8 XCDs.  Work items (range, tile) are
// numbered range-major and XCD x takes the x-th contiguous eighth of them,
// so the tiles that march a range side by side share one L2 and their
// x2 / x3 halo reads hit there.  The range length and the tile shape are a
// tuned variant (wd_tune_dirac); by default the ranges are as short as lets
// every work item be resident at once, and the tiles are LDS-staged bricks
// where they fit.
//
// LDS-staged form (brick tiles, FP64 and FP32 storage): at the start of each
// step the block copies the spinors of its brick's slice and of the brick's
// four side faces into LDS (each lane its own site and up to three face
// sites) and reads all six spatial neighbours from there, so a spinor's
// seven reads within a step no longer depend on it staying in L2; only the
// face sites, which the neighbouring bricks load in the same step, go
// through L2.
//
// Epilogue as in the single-parity hop: EPI 1 out = X + a H in, EPI 2
// out = X - Y + a H in (full fields), with an optional FP64 |out|^2.  XIN:
// X is the input field itself (D_W = 1 - kappa H), taken from the spinor
// already in registers.
#include <algorithm>

#include "wd_blas.h"
#include "wd_hop.h"

namespace wd {

namespace {

constexpr int DM_BS = 256;

struct KDirac {
  Geom g;
  const char *in;
  char *out;
  const char *X;
  const char *Y;
  const char *links[2];  // hop-link arrays of output parity 0 and 1
  size_t half;           // bytes per half field
  double a;
  double *partials;
  const int *skip;  // device flag: nothing to do when set
  int nsp;    // sites per time slice (L1 L2 L3)
  int nt;     // tiles of DM_BS spatial sites per slice
  int S;      // time slices per range
  int items;  // nt * number of ranges
  int per;    // work items per XCD
  int npad;   // padding slots per half field (zeroed)
  int n2;     // brick tiles: x2 rows per tile (0: tiles of consecutive sites)
  int n3;     // brick tiles: x3 planes per tile
  int nslot;  // LDS-staged form: staged sites per block (the brick and its four side faces)
};

// What a lane carries from one step to the next.
template <int P>
struct MarchCarry {
  cplx<RealOf<P>> acc[12];  // X + a (spatial + backward time hops) - Y of out(x, k)
  cplx<RealOf<P>> u4[6];    // U_{(x,k),4}: rows 0, 1
  cplx<RealOf<P>> gb[6];    // a U^dag_{(x,k),4} (projected psi(x,k)): the backward time hop of out(x, k+1)
};

// Lane constants: spatial neighbour offsets (checkerboard index deltas, the
// same on every slice), index and parity of the lane's site at x4 = 0.
struct MarchLane {
  int dn[6];  // x1+, x2+, x3+, x1-, x2-, x3-
  int i0;
  int par0;
};

__device__ __forceinline__ MarchLane march_lane(const Geom &g, int s) {
  MarchLane m;
  const int L1 = g.L[0], L2 = g.L[1], L3 = g.L[2];
  const int x1 = s % L1, r3 = s / L1, x2 = r3 % L2, x3 = r3 / L2;
  const int xp1 = (x1 + 1 == L1) ? 0 : x1 + 1, xm1 = (x1 == 0) ? L1 - 1 : x1 - 1;
  m.dn[0] = (xp1 >> 1) - (x1 >> 1);
  m.dn[3] = (xm1 >> 1) - (x1 >> 1);
  m.dn[1] = (x2 == L2 - 1) ? -(L2 - 1) * g.s2 : g.s2;
  m.dn[4] = (x2 == 0) ? (L2 - 1) * g.s2 : -g.s2;
  m.dn[2] = (x3 == L3 - 1) ? -(L3 - 1) * g.s3 : g.s3;
  m.dn[5] = (x3 == 0) ? (L3 - 1) * g.s3 : -g.s3;
  m.i0 = (x1 >> 1) + g.s2 * x2 + g.s3 * x3;
  m.par0 = (x1 + x2 + x3) & 1;
  return m;
}

// gb = U^dag (f h) for the backward time hop (projector sign B): h is the
// half of psi that (1 + B gamma_4) keeps, f = 2 a times the boundary factor.
template <int P, int B>
__device__ __forceinline__ void time_back(const cplx<RealOf<P>> (&u)[6], const cplx<RealOf<P>> (&half)[6],
                                          RealOf<P> f, cplx<RealOf<P>> (&gb)[6]) {
  using T = RealOf<P>;
  cplx<T> r2[3];
  rebuild_row2(u, r2);
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    cplx<T> v[3] = {f * half[3 * a], f * half[3 * a + 1], f * half[3 * a + 2]};
    cplx<T> y[3];
    su3_mul_dag(u, r2, v, y);
    gb[3 * a] = y[0];
    gb[3 * a + 1] = y[1];
    gb[3 * a + 2] = y[2];
  }
}

// Finishes out(x, k-1) = acc + U (f h) (forward time hop, sign F; h the half
// of psi(x, k) that the projector keeps, f = 2 a times the boundary factor)
// and stores it; returns its |out|^2 when NORM.
template <int P, int F, bool NORM>
__device__ __forceinline__ double time_fwd_store(const KDirac &k, cplx<RealOf<P>> (&acc)[12],
                                                 const cplx<RealOf<P>> (&u)[6], const cplx<RealOf<P>> (&half)[6],
                                                 RealOf<P> f, int p, size_t i) {
  using T = RealOf<P>;
  cplx<T> r2[3];
  rebuild_row2(u, r2);
  constexpr int o = F > 0 ? 0 : 6;  // the projector (1 + F gamma_4) keeps the upper (F > 0) or lower rows
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    cplx<T> v[3] = {f * half[3 * h], f * half[3 * h + 1], f * half[3 * h + 2]};
    cplx<T> y[3];
    su3_mul(u, r2, v, y);
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[o + 3 * h + c] = acc[o + 3 * h + c] + y[c];
  }
  char *out = k.out + (size_t)p * k.half;
  Spinor<P>::store(out, i, acc);
  double nrm = 0.0;
  if constexpr (NORM) {
    cplx<T> st[12];
    if constexpr (P == WD_F64 || P == WD_F32) {
#pragma unroll
      for (int q = 0; q < 12; ++q) st[q] = acc[q];
    } else {
      Spinor<P>::load(out, i, st);
    }
#pragma unroll
    for (int q = 0; q < 12; ++q) nrm += (double)st[q].re * st[q].re + (double)st[q].im * st[q].im;
  }
  return nrm;
}

// acc += a M (1 + S gamma_MU) psi_nb for a spatial hop: the projected half
// spinor is scaled by a before the link multiply (LDAG: M = u^dag).
template <int P, int MU, int S, bool LDAG>
__device__ __forceinline__ void hop_scaled(cplx<RealOf<P>> (&acc)[12], const char *in, int nb,
                                           const cplx<RealOf<P>> (&u)[6], RealOf<P> a) {
  using T = RealOf<P>;
  cplx<T> psi[12], h[6];
  Spinor<P>::load(in, nb, psi);
  project<MU, S>(psi, h);
#pragma unroll
  for (int c = 0; c < 6; ++c) h[c] = a * h[c];
  hop_term_h<P, MU, S, LDAG>(acc, h, u);
}

// Raw 16-byte packets of a stored spinor (FP64: 12, FP32: 6), in the
// order of the field layout; unpacked exactly as Spinor<P>::load does.
template <int P>
struct Raw;
template <>
struct Raw<WD_F64> {
  using V = v2d;
  static constexpr int N = 12;
  __device__ static void unpack(const V (&r)[N], cplx<double> (&s)[12]) {
#pragma unroll
    for (int c = 0; c < 12; ++c) s[c] = {r[c].x, r[c].y};
  }
};
template <>
struct Raw<WD_F32> {
  using V = v4f;
  static constexpr int N = 6;
  __device__ static void unpack(const V (&r)[N], cplx<float> (&s)[12]) {
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      s[2 * q] = {r[q].x, r[q].y};
      s[2 * q + 1] = {r[q].z, r[q].w};
    }
  }
};

template <int P>
__device__ __forceinline__ void raw_load(const char *base, int i, typename Raw<P>::V (&r)[Raw<P>::N]) {
  using V = typename Raw<P>::V;
  const V *q = (const V *)base + chunk_base<Raw<P>::N * 64>((size_t)i);
#pragma unroll
  for (int c = 0; c < Raw<P>::N; ++c) r[c] = q[64 * c];
}

// LDS: packet c of staged site `slot` at lds[c * nslot + slot] (consecutive
// lanes touch consecutive 16-byte words).
template <int P>
__device__ __forceinline__ void raw_to_lds(typename Raw<P>::V *lds, int nslot, int slot,
                                           const typename Raw<P>::V (&r)[Raw<P>::N]) {
#pragma unroll
  for (int c = 0; c < Raw<P>::N; ++c) lds[c * nslot + slot] = r[c];
}

// The staging plan of a lane in the LDS-staged form: its own slot is its
// thread index; the six spatial neighbours' slots; up to 3 face sites it
// stages (slot, checkerboard index and parity at x4 = 0).
struct MarchLds {
  int nsl[6];  // x1+, x2+, x3+, x1-, x2-, x3-
  int nh;
  int hslot[3], hi0[3], hpar0[3];
};

// Staged sites of a brick tile (L1 x n2 x n3 sites at x2 = b2 n2 + a2, x3 =
// b3 n3 + a3): slots 0..255 the brick, lane t = x1 + L1 (a2 + n2 a3); then
// the two x2 faces (a2 = -1, n2; 2 L1 n3 sites), then the two x3 faces
// (a3 = -1, n3; 2 L1 n2 sites).
__device__ __forceinline__ MarchLds march_lds_plan(const Geom &g, int n2, int n3, int b2, int b3, int tid) {
  MarchLds m;
  const int L1 = g.L[0], L2 = g.L[1], L3 = g.L[2];
  const int x1 = tid % L1, r = tid / L1, a2 = r % n2, a3 = r / n2;
  const int F2 = DM_BS, F3 = DM_BS + 2 * L1 * n3;
  auto own = [&](int y1, int c2, int c3) { return y1 + L1 * (c2 + n2 * c3); };
  m.nsl[0] = own(x1 + 1 == L1 ? 0 : x1 + 1, a2, a3);
  m.nsl[3] = own(x1 == 0 ? L1 - 1 : x1 - 1, a2, a3);
  m.nsl[1] = (a2 + 1 < n2) ? own(x1, a2 + 1, a3) : F2 + x1 + L1 * (a3 + n3);
  m.nsl[4] = (a2 > 0) ? own(x1, a2 - 1, a3) : F2 + x1 + L1 * a3;
  m.nsl[2] = (a3 + 1 < n3) ? own(x1, a2, a3 + 1) : F3 + x1 + L1 * (a2 + n2);
  m.nsl[5] = (a3 > 0) ? own(x1, a2, a3 - 1) : F3 + x1 + L1 * a2;
  const int nface = 2 * L1 * (n2 + n3);
  m.nh = 0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int h = tid + j * DM_BS;
    int y1 = 0, y2 = 0, y3 = 0;
    if (h < 2 * L1 * n3) {
      const int q = h / L1, c3 = q % n3, f = q / n3;
      y1 = h % L1;
      y2 = (b2 * n2 + (f ? n2 : -1) + L2) % L2;
      y3 = b3 * n3 + c3;
    } else {
      const int e = h - 2 * L1 * n3, q = e / L1, c2 = q % n2, f = q / n2;
      y1 = e % L1;
      y2 = b2 * n2 + c2;
      y3 = (b3 * n3 + (f ? n3 : -1) + L3) % L3;
    }
    m.hslot[j] = DM_BS + h;
    m.hi0[j] = (y1 >> 1) + g.s2 * y2 + g.s3 * y3;
    m.hpar0[j] = (y1 + y2 + y3) & 1;
    if (h < nface) m.nh = j + 1;
  }
  return m;
}

// acc += a M (1 + S gamma_MU) psi for a spatial hop whose neighbour spinor
// is staged in LDS.
template <int P, int MU, int S, bool LDAG>
__device__ __forceinline__ void hop_lds(cplx<RealOf<P>> (&acc)[12], const typename Raw<P>::V *lds, int nslot,
                                        int slot, const cplx<RealOf<P>> (&u)[6], RealOf<P> a) {
  using T = RealOf<P>;
  typename Raw<P>::V r[Raw<P>::N];
#pragma unroll
  for (int c = 0; c < Raw<P>::N; ++c) r[c] = lds[c * nslot + slot];
  cplx<T> psi[12], h[6];
  Raw<P>::unpack(r, psi);
  project<MU, S>(psi, h);
#pragma unroll
  for (int c = 0; c < 6; ++c) h[c] = a * h[c];
  hop_term_h<P, MU, S, LDAG>(acc, h, u);
}

// One step on slice t: finish out(x, t-1) (FIN), then build the carry for
// out(x, t) and the backward time hop of out(x, t+1).
template <int P, bool DAG, int EPI, bool XIN, bool NORM, bool FIN, bool LDS>
__device__ __forceinline__ double march_step(const KDirac &k, const MarchLane &m, int t, MarchCarry<P> &c,
                                             void *lds_raw, const MarchLds &pl) {
  using T = RealOf<P>;
  constexpr int F = DAG ? -1 : 1;
  constexpr int B = -F;
  const Geom &g = k.g;
  const int L4 = g.L[3];
  const int p = (m.par0 + t) & 1;
  const size_t i = (size_t)m.i0 + (size_t)t * g.s4;
  cplx<T> psi[12];
  if constexpr (LDS) {
    // stage slice t: the lane's own spinor and its share of the face sites
    using V = typename Raw<P>::V;
    V *lds = (V *)lds_raw;
    if constexpr (FIN) __syncthreads();  // the previous step has read the staged slice
    V r[Raw<P>::N];
    raw_load<P>(k.in + (size_t)p * k.half, (int)i, r);
    raw_to_lds<P>(lds, k.nslot, (int)threadIdx.x, r);
    Raw<P>::unpack(r, psi);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if (j < pl.nh) {
        V hr[Raw<P>::N];
        raw_load<P>(k.in + (size_t)((pl.hpar0[j] + t) & 1) * k.half, pl.hi0[j] + t * g.s4, hr);
        raw_to_lds<P>(lds, k.nslot, pl.hslot[j], hr);
      }
    }
  } else {
    Spinor<P>::load(k.in + (size_t)p * k.half, i, psi);
  }
  double nrm = 0.0;
  const T one = (T)1;
  if constexpr (FIN) {
    cplx<T> h[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) h[q] = psi[(F > 0 ? 0 : 6) + q];
    const T f = (T)2 * ((t - 1 == L4 - 1) ? (T)g.tbc : one) * (T)k.a;
    nrm = time_fwd_store<P, F, NORM>(k, c.acc, c.u4, h, f, 1 - p, i - g.s4);
  }
  // backward time hop received by out(x, t+1), from U_{(x,t),4}
  cplx<T> gb_next[6];
  Link<T>::template load<true>(k.links[p], 3, i, c.u4);
  {
    cplx<T> h[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) h[q] = psi[(B > 0 ? 0 : 6) + q];
    const T f = (T)2 * ((t == L4 - 1) ? (T)g.tbc : one) * (T)k.a;
    time_back<P, B>(c.u4, h, f, gb_next);
  }
  // out(x, t) starts from the epilogue terms X - Y, so that the own spinor
  // is dead before the spatial hops; each hop then adds a times its term
  // (the projected half spinor is scaled by a before the link multiply)
  cplx<T> acc[12];
  if constexpr (XIN) {
#pragma unroll
    for (int q = 0; q < 12; ++q) acc[q] = psi[q];
  } else if constexpr (EPI >= 1) {
    Spinor<P>::load(k.X + (size_t)p * k.half, i, acc);
  } else {
#pragma unroll
    for (int q = 0; q < 12; ++q) acc[q] = {(T)0, (T)0};
  }
  if constexpr (EPI == 2) {
    cplx<T> y[12];
    Spinor<P>::load(k.Y + (size_t)p * k.half, i, y);
#pragma unroll
    for (int q = 0; q < 12; ++q) acc[q] = acc[q] - y[q];
  }
  reconstruct_add<3, B>(acc, c.gb);  // the backward time hop, formed one step earlier
  const T a = (T)k.a;
  const char *inn = k.in + (size_t)(1 - p) * k.half;
  const char *Lo = k.links[p], *Ln = k.links[1 - p];
  // forward and backward hop of each direction back to back: a spatial link
  // is read by its owner and by the neighbour it points to close together
  cplx<T> u[6];
  if constexpr (LDS) {
    using V = typename Raw<P>::V;
    const V *lds = (const V *)lds_raw;
    __syncthreads();  // slice t is staged
    Link<T>::template load<false>(Lo, 0, i, u);
    hop_lds<P, 0, F, false>(acc, lds, k.nslot, pl.nsl[0], u, a);
    Link<T>::template load<false>(Ln, 0, i + m.dn[3], u);
    hop_lds<P, 0, B, true>(acc, lds, k.nslot, pl.nsl[3], u, a);
    Link<T>::template load<false>(Lo, 1, i, u);
    hop_lds<P, 1, F, false>(acc, lds, k.nslot, pl.nsl[1], u, a);
    Link<T>::template load<false>(Ln, 1, i + m.dn[4], u);
    hop_lds<P, 1, B, true>(acc, lds, k.nslot, pl.nsl[4], u, a);
    Link<T>::template load<false>(Lo, 2, i, u);
    hop_lds<P, 2, F, false>(acc, lds, k.nslot, pl.nsl[2], u, a);
    Link<T>::template load<false>(Ln, 2, i + m.dn[5], u);
    hop_lds<P, 2, B, true>(acc, lds, k.nslot, pl.nsl[5], u, a);
  } else {
    Link<T>::template load<false>(Lo, 0, i, u);
    hop_scaled<P, 0, F, false>(acc, inn, (int)i + m.dn[0], u, a);
    Link<T>::template load<false>(Ln, 0, i + m.dn[3], u);
    hop_scaled<P, 0, B, true>(acc, inn, (int)i + m.dn[3], u, a);
    Link<T>::template load<false>(Lo, 1, i, u);
    hop_scaled<P, 1, F, false>(acc, inn, (int)i + m.dn[1], u, a);
    Link<T>::template load<false>(Ln, 1, i + m.dn[4], u);
    hop_scaled<P, 1, B, true>(acc, inn, (int)i + m.dn[4], u, a);
    Link<T>::template load<false>(Lo, 2, i, u);
    hop_scaled<P, 2, F, false>(acc, inn, (int)i + m.dn[2], u, a);
    Link<T>::template load<false>(Ln, 2, i + m.dn[5], u);
    hop_scaled<P, 2, B, true>(acc, inn, (int)i + m.dn[5], u, a);
  }
#pragma unroll
  for (int q = 0; q < 12; ++q) c.acc[q] = acc[q];
#pragma unroll
  for (int q = 0; q < 6; ++q) c.gb[q] = gb_next[q];
  return nrm;
}

template <int P, bool DAG, int EPI, bool XIN, bool NORM, bool LDS>
__global__ __launch_bounds__(DM_BS) void k_dirac_march(KDirac k) {
  extern __shared__ __align__(16) unsigned char dm_lds[];
  using T = RealOf<P>;
  constexpr int F = DAG ? -1 : 1;
  constexpr int B = -F;
  if (k.skip && *k.skip) return;
  const int b = (int)blockIdx.x, q = b >> 3;
  const int item = (b & 7) * k.per + q;
  double nrm = 0.0;
  if (q < k.per && item < k.items) {
    const int tile = item % k.nt, r = item / k.nt;
    int s = tile * DM_BS + (int)threadIdx.x;
    MarchLds pl{};
    if (k.n2 > 0) {
      // brick tile of L1 x n2 x n3 sites: half of its x3 neighbours and all
      // but 2 / n2 of its x2 neighbours are its own
      const int L1 = k.g.L[0], nb2 = k.g.L[1] / k.n2;
      const int tid = (int)threadIdx.x, rr = tid / L1;
      const int x2 = (tile % nb2) * k.n2 + rr % k.n2, x3 = (tile / nb2) * k.n3 + rr / k.n2;
      s = tid % L1 + L1 * (x2 + k.g.L[1] * x3);
      if constexpr (LDS) pl = march_lds_plan(k.g, k.n2, k.n3, tile % nb2, tile / nb2, tid);
    }
    if (r == 0) {
      // padding slots of both halves stay zero
      cplx<T> z[12];
#pragma unroll
      for (int j = 0; j < 12; ++j) z[j] = {(T)0, (T)0};
      for (int j = s; j < k.npad; j += k.nt * DM_BS) {
        Spinor<P>::store(k.out, (size_t)k.g.vh + j, z);
        Spinor<P>::store(k.out + k.half, (size_t)k.g.vh + j, z);
      }
    }
    if (s < k.nsp) {
      const Geom &g = k.g;
      const int L4 = g.L[3];
      const MarchLane m = march_lane(g, s);
      const int t0 = r * k.S, t1 = min(t0 + k.S, L4);
      MarchCarry<P> c;
      {
        // the backward time hop that out(x, t0) receives from slice t0 - 1
        const int tp = (t0 == 0) ? L4 - 1 : t0 - 1;
        const int p = (m.par0 + tp) & 1;
        const size_t i = (size_t)m.i0 + (size_t)tp * g.s4;
        cplx<T> h[6], u[6];
        Spinor<P>::template load_half<(B < 0)>(k.in + (size_t)p * k.half, i, h);
        Link<T>::template load<true>(k.links[p], 3, i, u);
        time_back<P, B>(u, h, (T)2 * ((tp == L4 - 1) ? (T)g.tbc : (T)1) * (T)k.a, c.gb);
      }
      nrm += march_step<P, DAG, EPI, XIN, NORM, false, LDS>(k, m, t0, c, dm_lds, pl);
#pragma unroll 1
      for (int t = t0 + 1; t < t1; ++t) nrm += march_step<P, DAG, EPI, XIN, NORM, true, LDS>(k, m, t, c, dm_lds, pl);
      {
        // the forward time hop of out(x, t1 - 1) from slice t1
        const int te = (t1 == L4) ? 0 : t1;
        const int p = (m.par0 + te) & 1;
        cplx<T> h[6];
        Spinor<P>::template load_half<(F < 0)>(k.in + (size_t)p * k.half, (size_t)m.i0 + (size_t)te * g.s4, h);
        const T f = (T)2 * ((t1 - 1 == L4 - 1) ? (T)g.tbc : (T)1) * (T)k.a;
        nrm += time_fwd_store<P, F, NORM>(k, c.acc, c.u4, h, f, 1 - p, (size_t)m.i0 + (size_t)(t1 - 1) * g.s4);
      }
    }
  }
  if constexpr (NORM) {
    double v[1] = {nrm};
    block_sum_store<1>(v, k.partials, gridDim.x, blockIdx.x);
  }
}

template <int P, bool DAG, bool LDS>
void launch_p(const KDirac &k, int epi, bool xin, bool norm, unsigned nblk, size_t lds, hipStream_t st) {
#define WD_DR(E, XI, N)                    \
  if (epi == E && xin == XI && norm == N) \
    hipLaunchKernelGGL((k_dirac_march<P, DAG, E, XI, N, LDS>), dim3(nblk), dim3(DM_BS), lds, st, k);
  WD_DR(0, false, false) WD_DR(1, false, false) WD_DR(2, false, false)
  WD_DR(1, true, false) WD_DR(2, true, false)
  WD_DR(0, false, true) WD_DR(1, false, true) WD_DR(2, false, true)
  WD_DR(1, true, true) WD_DR(2, true, true)
#undef WD_DR
}

struct MarchGrid {
  int nsp, nt, S, items, per, n2, n3;
};

// Brick tiles of L1 x n2 x 2 sites (L1 n2 2 = 256) fit when n2 divides L2
// and L3 is even; n2 = 0 if not.
int march_brick_n2(const Geom &g) {
  if (DM_BS % (2 * g.L[0]) != 0) return 0;
  const int n2 = DM_BS / (2 * g.L[0]);
  return (g.L[1] % n2 == 0 && g.L[2] % 2 == 0) ? n2 : 0;
}

// Staged sites and LDS bytes per block of the LDS-staged form (the brick
// and its four side faces; FP64 12, FP32 6 packets of 16 bytes per site).
int march_nslot(const Geom &g, int n2) { return DM_BS + 2 * g.L[0] * (n2 + 2); }
size_t march_lds_bytes(const Geom &g, wd_prec prec) {
  const int n2 = march_brick_n2(g);
  return n2 ? (size_t)march_nslot(g, n2) * (prec == WD_F64 ? 12 : 6) * 16 : 0;
}

// tile: 2 = brick tiles, 3 = brick tiles staged in LDS (where bricks fit),
// 0 = 256 consecutive spatial sites.
// S > 0: time slices per range (at most L4); S = 0: the smallest of 8, 16,
// 32, ... for which every work item is resident at once (capacity =
// resident blocks per CU x CUs), so that the tiles marching a range side by
// side run together.
MarchGrid march_grid(const Geom &g, int S, int tile, int capacity) {
  MarchGrid m;
  m.nsp = g.L[0] * g.L[1] * g.L[2];
  m.n2 = tile >= 2 ? march_brick_n2(g) : 0;
  m.n3 = m.n2 ? 2 : 0;
  m.nt = m.n2 ? (g.L[1] / m.n2) * (g.L[2] / m.n3) : (m.nsp + DM_BS - 1) / DM_BS;
  if (S > 0) {
    m.S = std::min(S, g.L[3]);
  } else {
    m.S = std::min(8, g.L[3]);
    while (m.S < g.L[3] && (long)m.nt * ((g.L[3] + m.S - 1) / m.S) > capacity) m.S *= 2;
    m.S = std::min(m.S, g.L[3]);
  }
  m.items = m.nt * ((g.L[3] + m.S - 1) / m.S);
  m.per = (m.items + 7) / 8;
  return m;
}

template <int P, bool LDS>
int march_blocks_per_cu(size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_dirac_march<P, false, 1, true, false, LDS>, DM_BS, lds) !=
          hipSuccess ||
      n < 1)
    n = 1;
  return n;
}

int march_capacity(const wd_gauge *g, wd_prec prec) {
  const int bpc = (g->dirac_tile[prec] == 3 && prec <= WD_F32) ? g->dirac_bpc_lds[prec] : g->dirac_bpc[prec];
  return std::max(bpc, 1) * std::max(g->n_cu, 1);
}

MarchGrid march_grid_of(const wd_gauge *g, wd_prec prec) {
  return march_grid(g->geom, g->dirac_slices[prec], g->dirac_tile[prec], march_capacity(g, prec));
}

}  // namespace

bool dirac_variant_ok(const wd_gauge *g, wd_prec prec, int slices, int tile) {
  const Geom &G = g->geom;
  if (slices < 0 || slices > G.L[3]) return false;
  if (tile == 0) return true;
  if (tile == 2) return march_brick_n2(G) > 0;
  if (tile == 3)
    return march_brick_n2(G) > 0 && (prec == WD_F64 || prec == WD_F32) &&
           march_lds_bytes(G, prec) <= (size_t)g->lds_per_block;
  return false;
}

wd_status dirac_init(wd_gauge *g) {
  // default tiles: bricks staged in LDS where they fit (FP64, FP32), else bricks, else consecutive sites
  for (int p = 0; p < 4; ++p) {
    g->dirac_slices[p] = 0;
    g->dirac_tile[p] = march_brick_n2(g->geom) ? 2 : 0;
  }
  g->dirac_bpc[WD_F64] = march_blocks_per_cu<WD_F64, false>(0);
  g->dirac_bpc[WD_F32] = march_blocks_per_cu<WD_F32, false>(0);
  g->dirac_bpc[WD_F16] = march_blocks_per_cu<WD_F16, false>(0);
  g->dirac_bpc[WD_BF16] = march_blocks_per_cu<WD_BF16, false>(0);
  g->dirac_bpc_lds[WD_F64] = g->dirac_bpc_lds[WD_F32] = 0;
  if (dirac_variant_ok(g, WD_F64, 0, 3))
    g->dirac_bpc_lds[WD_F64] = march_blocks_per_cu<WD_F64, true>(march_lds_bytes(g->geom, WD_F64));
  if (dirac_variant_ok(g, WD_F32, 0, 3))
    g->dirac_bpc_lds[WD_F32] = march_blocks_per_cu<WD_F32, true>(march_lds_bytes(g->geom, WD_F32));
  for (int p = 0; p < 2; ++p)
    if (g->dirac_bpc_lds[p] > 0) g->dirac_tile[p] = 3;
  return WD_OK;
}

bool dirac_fills_device(const wd_gauge *g, wd_prec prec) {
  const int cap = march_capacity(g, prec);
  return 2 * march_grid_of(g, prec).items >= cap;
}

wd_status launch_dirac(const wd_gauge *g, wd_prec prec, const DiracArgs &a, hipStream_t st) {
  if (a.Y && !a.X) return set_error(WD_ERR_ARG, "dirac epilogue: Y given without X");
  const bool norm = a.norm_out != nullptr;
  if (norm && !a.red.partials) return set_error(WD_ERR_ARG, "dirac norm: no reduction buffer");
  KDirac k{};
  k.g = g->geom;
  k.in = (const char *)a.in;
  k.out = (char *)a.out;
  k.X = (const char *)a.X;
  k.Y = (const char *)a.Y;
  const bool f64 = prec == WD_F64;
  const char *lk = (const char *)(f64 ? g->links64 : g->links32);
  const size_t lp = link_parity_bytes(g->geom, f64);
  k.links[0] = lk;
  k.links[1] = lk + lp;
  k.half = half_bytes(g->geom, prec);
  k.a = a.a;
  k.partials = a.red.partials;
  k.skip = a.skip;
  if ((int)prec < 0 || (int)prec > 3) return set_error(WD_ERR_PREC, "dirac: unknown precision %d", (int)prec);
  const MarchGrid mg = march_grid_of(g, prec);
  k.nsp = mg.nsp;
  k.nt = mg.nt;
  k.S = mg.S;
  k.items = mg.items;
  k.per = mg.per;
  k.npad = g->geom.vpad - g->geom.vh;
  k.n2 = mg.n2;
  k.n3 = mg.n3;
  const bool staged = g->dirac_tile[prec] == 3;
  if (staged && !dirac_variant_ok(g, prec, g->dirac_slices[prec], 3))
    return set_error(WD_ERR_ARG, "dirac: the LDS-staged variant does not fit this lattice / precision");
  k.nslot = staged ? march_nslot(g->geom, mg.n2) : 0;
  const size_t lds = staged ? march_lds_bytes(g->geom, prec) : 0;
  const int epi = a.Y ? 2 : (a.X ? 1 : 0);
  const bool xin = a.X && a.X == a.in;
  const unsigned nblk = 8u * (unsigned)mg.per;
  // the reduction buffers hold at least this many partials (sized for the hop and level-1 grids)
  if (norm && nblk > std::max(dslash_grid_blocks(g), BLAS_MAX_BLOCKS))
    return set_error(WD_ERR_ARG, "dirac norm: %u blocks exceed the reduction buffer", nblk);
#define WD_DP(PR, L)                                                           \
  if (a.dagger) launch_p<PR, true, L>(k, epi, xin, norm, nblk, lds, st);        \
  else launch_p<PR, false, L>(k, epi, xin, norm, nblk, lds, st);
  switch (prec) {
    case WD_F64:
      if (staged) { WD_DP(WD_F64, true) } else { WD_DP(WD_F64, false) }
      break;
    case WD_F32:
      if (staged) { WD_DP(WD_F32, true) } else { WD_DP(WD_F32, false) }
      break;
    case WD_F16: WD_DP(WD_F16, false) break;
    case WD_BF16: WD_DP(WD_BF16, false) break;
    default: return set_error(WD_ERR_PREC, "dirac: unknown precision %d", (int)prec);
  }
#undef WD_DP
  WD_TRY(hip_check(hipGetLastError(), "dirac launch"));
  if (norm) return launch_finish_sums(k.partials, nblk, 1, a.norm_out, 1, a.norm_accumulate, a.skip, 1, st);
  return WD_OK;
}

}  // namespace wd
