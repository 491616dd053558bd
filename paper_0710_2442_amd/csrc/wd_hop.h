// Per-site Wilson hop (Eq. 3 on one checkerboard), shared by the
// single-lattice, multi-RHS and batched multi-lattice kernels.
#pragma once

#include "wd_device.h"

namespace wd {

template <int P>
using RealOf = typename Spinor<P>::real;

struct KDslash {
  Geom g;
  const char *in;
  char *out;
  const char *X;
  const char *Y;
  const char *links;  // hop-link arrays of this output parity
  double a;
  int parity;
  int norm_accumulate;
  double *norm_out;
  const int *skip;
  double *partials;
  // block -> tile mapping (see tile_of)
  int groups;           // 0: linear; G > 0: G contiguous regions per time slice
  int tiles_per_slice;  // tiles (blocks) per time slice of one parity
  int occ;              // register-budget variant (0 or 4), host side only
  int nt_store;         // 1: streaming output stores; 0: cached stores
  int preload;          // 1: load all 8 links before the first hop (FP32 arithmetic only), host side
  int stage;            // 1: stage the tile's input spinors in LDS (FP64, FP32), host side
  int spl;              // sites per lane along x4 (1, 2, 4): lane covers tiles t, t + T, ... of consecutive slices
};

// Workgroups are dispatched round-robin over the XCDs (8 on MI355X), each
// with its own L2.  groups = G > 0: block b goes to region b % G and the
// blocks of one region walk its tiles slice by slice in time order, so a
// region's neighbour spinors (x1..x3 inside the slice, x4 one slice away)
// are fetched into one L2 and re-read from there.  Requires
// tiles_per_slice % G == 0.  groups = -X: the time slices are cut into X
// contiguous ranges and block b walks range b % X in time order; with X = 8
// each XCD sweeps its own block of slices, so the spatial neighbours (same
// slice) and the time neighbours (the slices before and after) of a site are
// all re-read from that XCD's L2.  Requires L4 % X == 0.  Both need
// gridDim.x == tiles_per_slice * L4.
__device__ __forceinline__ int tile_of(const KDslash &k, int b) {
  if (k.groups == 0) return b;
  const int T = k.tiles_per_slice;
  if (k.groups <= -100) {
    // box order: dispatch lane x = b % 8 (one per XCD) owns the box of x3
    // planes [bx * P, bx * P + P) and time slices [bt * S, bt * S + S),
    // nx3 = -groups - 100 boxes along x3 and 8 / nx3 along x4, and walks it
    // slice by slice, plane by plane, so that every neighbour of a site but
    // those across a box face is fetched into that XCD's L2, and the next
    // slice's sites (the time neighbours) are at most one box slice away.
    const int nx3 = -k.groups - 100;
    const int P = k.g.L[2] / nx3, S = k.g.L[3] / (8 / nx3);
    const int tpp = T / k.g.L[2];  // tiles per x3 plane
    const int x = b & 7, q = b >> 3;
    const int bx = x % nx3, bt = x / nx3;
    const int s = q / (P * tpp), pl = (q / tpp) % P, tp = q % tpp;
    return ((bt * S + s) * k.g.L[2] + bx * P + pl) * tpp + tp;
  }
  if (k.groups < 0) {
    const int X = -k.groups;
    const int x = b % X, q = b / X;
    const int per = k.g.L[3] / X;  // slices per range
    return (x * per + q / T) * T + (q % T);
  }
  const int G = k.groups;
  const int per = T / G;
  const int x = b % G, q = b / G;
  return (q / per) * T + x * per + (q % per);
}
__device__ __forceinline__ int tile_of(const KDslash &k) { return tile_of(k, (int)blockIdx.x); }


// Site coordinates of checkerboard index i on parity p.
struct Coords {
  int x1, x2, x3, x4, rest;
};
__device__ __forceinline__ Coords coords_of(const Geom &g, int i, int parity) {
  Coords c;
  const int x1h = i % g.L1h;
  c.rest = i / g.L1h;
  c.x2 = c.rest % g.L[1];
  const int r2 = c.rest / g.L[1];
  c.x3 = r2 % g.L[2];
  c.x4 = r2 / g.L[2];
  c.x1 = 2 * x1h + ((parity + c.x2 + c.x3 + c.x4) & 1);
  return c;
}

// Checkerboard indices of the 8 neighbours, in hop order
// (x1+, x2+, x3+, x4+, x1-, x2-, x3-, x4-).
__device__ __forceinline__ void neighbours(const Geom &g, const Coords &c, int i, int (&nb)[8]) {
  const int xp1 = (c.x1 + 1 == g.L[0]) ? 0 : c.x1 + 1;
  const int xm1 = (c.x1 == 0) ? g.L[0] - 1 : c.x1 - 1;
  nb[0] = (xp1 >> 1) + g.L1h * c.rest;
  nb[4] = (xm1 >> 1) + g.L1h * c.rest;
  nb[1] = i + ((c.x2 == g.L[1] - 1) ? -(g.L[1] - 1) * g.s2 : g.s2);
  nb[5] = i + ((c.x2 == 0) ? (g.L[1] - 1) * g.s2 : -g.s2);
  nb[2] = i + ((c.x3 == g.L[2] - 1) ? -(g.L[2] - 1) * g.s3 : g.s3);
  nb[6] = i + ((c.x3 == 0) ? (g.L[2] - 1) * g.s3 : -g.s3);
  nb[3] = i + ((c.x4 == g.L[3] - 1) ? -(g.L[3] - 1) * g.s4 : g.s4);
  nb[7] = i + ((c.x4 == 0) ? (g.L[3] - 1) * g.s4 : -g.s4);
}

// One hop: acc += M (1 + S gamma_MU) psi_nb, M = the hop link u (rows 0, 1;
// row 2 rebuilt).  Time hops (MU = 3) read only the half of the neighbour
// spinor that their projector keeps (see the spin basis in wd_device.h).
// LDAG: multiply by u^dag instead of u (u holds the rows of the link that
// the neighbour stores as its forward link).
template <int P, int MU, int S, bool LDAG = false>
__device__ __forceinline__ void hop_term_h(cplx<RealOf<P>> (&acc)[12], const cplx<RealOf<P>> (&h)[6],
                                           const cplx<RealOf<P>> (&u)[6]);

template <int P, int MU, int S, bool LDAG = false>
__device__ __forceinline__ void hop_term_u(cplx<RealOf<P>> (&acc)[12], const char *in, int nb,
                                           const cplx<RealOf<P>> (&u)[6], RealOf<P> sign) {
  using T = RealOf<P>;
  cplx<T> h[6];
  if constexpr (MU == 3) {
    Spinor<P>::template load_half<(S < 0)>(in, nb, h);
    const T f = (T)2 * sign;
#pragma unroll
    for (int c = 0; c < 6; ++c) h[c] = f * h[c];
  } else {
    cplx<T> psi[12];
    Spinor<P>::load(in, nb, psi);
    project<MU, S>(psi, h);
  }
  hop_term_h<P, MU, S, LDAG>(acc, h, u);
}

// The same for a spatial hop (MU < 3) whose neighbour spinor is already in
// registers (read from LDS by the staged kernel).
template <int P, int MU, int S>
__device__ __forceinline__ void hop_term_psi(cplx<RealOf<P>> (&acc)[12], const cplx<RealOf<P>> (&psi)[12],
                                             const cplx<RealOf<P>> (&u)[6]) {
  static_assert(MU < 3, "time hops read half spinors");
  cplx<RealOf<P>> h[6];
  project<MU, S>(psi, h);
  hop_term_h<P, MU, S>(acc, h, u);
}

// acc += reconstruct(M h): the projected half spinor h times the link.
template <int P, int MU, int S, bool LDAG>
__device__ __forceinline__ void hop_term_h(cplx<RealOf<P>> (&acc)[12], const cplx<RealOf<P>> (&h)[6],
                                           const cplx<RealOf<P>> (&u)[6]) {
  using T = RealOf<P>;
  cplx<T> r2[3];
  rebuild_row2(u, r2);
  cplx<T> g[6];
  {
    cplx<T> v[3] = {h[0], h[1], h[2]};
    cplx<T> y[3];
    if constexpr (LDAG) su3_mul_dag(u, r2, v, y);
    else su3_mul(u, r2, v, y);
    g[0] = y[0]; g[1] = y[1]; g[2] = y[2];
  }
  {
    cplx<T> v[3] = {h[3], h[4], h[5]};
    cplx<T> y[3];
    if constexpr (LDAG) su3_mul_dag(u, r2, v, y);
    else su3_mul(u, r2, v, y);
    g[3] = y[0]; g[4] = y[1]; g[5] = y[2];
  }
  reconstruct_add<MU, S>(acc, g);
}

// The same hop with the link loaded from the hop-link array (direction d).
template <int P, int MU, int S>
__device__ __forceinline__ void hop_term(cplx<RealOf<P>> (&acc)[12], const char *in, int nb,
                                         const char *links, int d, size_t i, RealOf<P> sign) {
  cplx<RealOf<P>> u[6];
  Link<RealOf<P>>::load(links, d, i, u);
  hop_term_u<P, MU, S>(acc, in, nb, u, sign);
}

// The 8 hops of site i with its links already in registers: u[d] for hop
// direction d (x1+, x2+, x3+, x4+, x1-, x2-, x3-, x4-).
template <int P, bool DAG>
__device__ __forceinline__ void hop_all_u(const char *in, const int (&nb)[8], const cplx<RealOf<P>> (&u)[8][6],
                                          RealOf<P> sf, RealOf<P> sb, cplx<RealOf<P>> (&acc)[12]) {
  using T = RealOf<P>;
  const T one = (T)1;
  constexpr int F = DAG ? -1 : 1;
  constexpr int B = -F;
#pragma unroll
  for (int c2 = 0; c2 < 12; ++c2) acc[c2] = {(T)0, (T)0};
  hop_term_u<P, 0, F>(acc, in, nb[0], u[0], one);
  hop_term_u<P, 1, F>(acc, in, nb[1], u[1], one);
  hop_term_u<P, 2, F>(acc, in, nb[2], u[2], one);
  hop_term_u<P, 3, F>(acc, in, nb[3], u[3], sf);
  hop_term_u<P, 0, B>(acc, in, nb[4], u[4], one);
  hop_term_u<P, 1, B>(acc, in, nb[5], u[5], one);
  hop_term_u<P, 2, B>(acc, in, nb[6], u[6], one);
  hop_term_u<P, 3, B>(acc, in, nb[7], u[7], sb);
}

template <int P, bool DAG>
__device__ __forceinline__ void hop_all(const KDslash &k, int i, cplx<RealOf<P>> (&acc)[12]) {
  using T = RealOf<P>;
  const Coords c = coords_of(k.g, i, k.parity);
  int nb[8];
  neighbours(k.g, c, i, nb);
  const T one = (T)1;
  const T sf = (c.x4 == k.g.L[3] - 1) ? (T)k.g.tbc : one;
  const T sb = (c.x4 == 0) ? (T)k.g.tbc : one;
  constexpr int F = DAG ? -1 : 1;  // forward hop projector (1 + F gamma)
  constexpr int B = -F;            // backward hop projector (1 + B gamma)
  const char *L = k.links;
#pragma unroll
  for (int c2 = 0; c2 < 12; ++c2) acc[c2] = {(T)0, (T)0};
  hop_term<P, 0, F>(acc, k.in, nb[0], L, 0, i, one);
  hop_term<P, 1, F>(acc, k.in, nb[1], L, 1, i, one);
  hop_term<P, 2, F>(acc, k.in, nb[2], L, 2, i, one);
  hop_term<P, 3, F>(acc, k.in, nb[3], L, 3, i, sf);
  hop_term<P, 0, B>(acc, k.in, nb[4], L, 4, i, one);
  hop_term<P, 1, B>(acc, k.in, nb[5], L, 5, i, one);
  hop_term<P, 2, B>(acc, k.in, nb[6], L, 6, i, one);
  hop_term<P, 3, B>(acc, k.in, nb[7], L, 7, i, sb);
}

// The 8 hops of site i with all 8 links loaded first: 48 (FP64) or 24
// (FP32) independent 16-byte loads in flight per lane before any arithmetic,
// at the cost of holding the links in registers.
template <int P, bool DAG>
__device__ __forceinline__ void hop_all_preload(const KDslash &k, int i, cplx<RealOf<P>> (&acc)[12]) {
  using T = RealOf<P>;
  const Coords c = coords_of(k.g, i, k.parity);
  int nb[8];
  neighbours(k.g, c, i, nb);
  const T sf = (c.x4 == k.g.L[3] - 1) ? (T)k.g.tbc : (T)1;
  const T sb = (c.x4 == 0) ? (T)k.g.tbc : (T)1;
  cplx<T> u[8][6];
#pragma unroll
  for (int d = 0; d < 8; ++d) Link<T>::load(k.links, d, i, u[d]);
  hop_all_u<P, DAG>(k.in, nb, u, sf, sb, acc);
}

// Neighbour spinors staged in LDS by a block whose tile is k whole x1 rows
// of one x3 plane (k | L2, k >= 2) or whole planes.  Slots 0 .. n-1 are the
// tile's own input sites t0 .. t0+n-1, slots n .. n+L1h-1 the x1 row before
// the tile's first row (its x2 - 1 neighbour row, wrapping in the plane)
// starting at site lo, and slots n+L1h .. n+2 L1h-1 the row after its last
// row starting at site hi: every x1 and x2 neighbour of the tile's output
// sites is one of these.  A slot holds the whole input spinor (the four x1
// and x2 hops project it four different ways) as 16-byte packets, packet-
// major: packet q (complex numbers qK .. qK+K-1, K = 16 / sizeof(cplx<T>))
// of slot s is packet q * ns + s, ns = n + 2 L1h.  Lanes that read one packet
// of consecutive slots touch consecutive 16-byte words, so the layout needs
// no padding against bank conflicts: 192 B per slot in FP64, 96 B in FP32.
template <class T>
struct __align__(16) StagePacket {
  cplx<T> v[16 / sizeof(cplx<T>)];
};
template <class T>
struct Stage {
  const cplx<T> *lds;
  int t0, n, lo, hi, l1h, ns;
};

// (every candidate computed, then selected: no branches, which would cut the
// hop into basic blocks the scheduler cannot interleave)
template <class T>
__device__ __forceinline__ int stage_slot(const Stage<T> &sv, int nb) {
  const int s = nb - sv.t0;
  const int l = nb - sv.lo;
  const int in_lo = sv.n + l;
  const int in_hi = sv.n + sv.l1h + (nb - sv.hi);
  int r = ((unsigned)l < (unsigned)sv.l1h) ? in_lo : in_hi;
  r = ((unsigned)s < (unsigned)sv.n) ? s : r;
  return r;
}

// psi into slot s of a stage of ns slots.
template <class T>
__device__ __forceinline__ void stage_store(cplx<T> *lds, int s, int ns, const cplx<T> (&psi)[12]) {
  constexpr int K = 16 / sizeof(cplx<T>);
  StagePacket<T> *p = (StagePacket<T> *)lds + s;
#pragma unroll
  for (int q = 0; q < 12 / K; ++q) {
    StagePacket<T> w;
#pragma unroll
    for (int j = 0; j < K; ++j) w.v[j] = psi[q * K + j];
    p[(size_t)q * ns] = w;
  }
}

// The spinor of slot `slot`.
template <class T>
__device__ __forceinline__ void stage_load(const Stage<T> &sv, int slot, cplx<T> (&psi)[12]) {
  constexpr int K = 16 / sizeof(cplx<T>);
  const StagePacket<T> *p = (const StagePacket<T> *)sv.lds + slot;
#pragma unroll
  for (int q = 0; q < 12 / K; ++q) {
    const StagePacket<T> w = p[(size_t)q * sv.ns];
#pragma unroll
    for (int j = 0; j < K; ++j) psi[q * K + j] = w.v[j];
  }
}

// A spatial hop (x1 or x2) with the neighbour's projection from the staged
// tile: the same values as projected from memory, so the result is bitwise
// that of hop_term.
template <int P, int MU, int S>
__device__ __forceinline__ void staged_term(cplx<RealOf<P>> (&acc)[12], const KDslash &k, const Stage<RealOf<P>> &sv,
                                            int nb, int d, size_t i) {
  using T = RealOf<P>;
  static_assert(MU < 2, "x1 and x2 hops only");
  cplx<T> u[6];
  Link<T>::load(k.links, d, i, u);
  cplx<T> psi[12];
  stage_load(sv, stage_slot(sv, nb), psi);
  hop_term_psi<P, MU, S>(acc, psi, u);
  // FP64: one hop at a time (started all at once, the hops' operands exceed
  // the registers); FP32 keeps the early loads, which hide more latency
  if constexpr (P == WD_F64) __builtin_amdgcn_sched_barrier(0);
}

// The same with the link already in registers.
template <int P, int MU, int S>
__device__ __forceinline__ void staged_term_u(cplx<RealOf<P>> (&acc)[12], const Stage<RealOf<P>> &sv, int nb,
                                              const cplx<RealOf<P>> (&u)[6]) {
  using T = RealOf<P>;
  cplx<T> psi[12];
  stage_load(sv, stage_slot(sv, nb), psi);
  hop_term_psi<P, MU, S>(acc, psi, u);
}

// A time hop on a half spinor h already loaded (load_half of the hop's
// projector), the same arithmetic as hop_term_u's time path.
template <int P, int S>
__device__ __forceinline__ void hop_term_x4(cplx<RealOf<P>> (&acc)[12], const cplx<RealOf<P>> (&hraw)[6],
                                            const cplx<RealOf<P>> (&u)[6], RealOf<P> sign) {
  using T = RealOf<P>;
  const T f = (T)2 * sign;
  cplx<T> h[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) h[c] = f * hraw[c];
  hop_term_h<P, 3, S>(acc, h, u);
}

// The 8 hops with the x1 and x2 neighbours read from the staged tile, the x3
// and x4 neighbours from memory.  Same hop order and arithmetic as hop_all.
// FP32: every link and every neighbour in memory is loaded before the first
// hop (the loads in flight hide more latency); FP64 takes one hop at a time
// (its operands would not fit the registers all at once).
template <int P, bool DAG>
__device__ __forceinline__ void hop_all_staged(const KDslash &k, int i, const Stage<RealOf<P>> &sv,
                                               cplx<RealOf<P>> (&acc)[12]) {
  using T = RealOf<P>;
  const Coords c = coords_of(k.g, i, k.parity);
  int nb[8];
  neighbours(k.g, c, i, nb);
  const T one = (T)1;
  const T sf = (c.x4 == k.g.L[3] - 1) ? (T)k.g.tbc : one;
  const T sb = (c.x4 == 0) ? (T)k.g.tbc : one;
  constexpr int F = DAG ? -1 : 1;
  constexpr int B = -F;
  const char *L = k.links;
  if constexpr (P == WD_F32) {
    cplx<T> u[8][6];
#pragma unroll
    for (int d = 0; d < 8; ++d) Link<T>::load(L, d, i, u[d]);
    cplx<T> p2f[12], p2b[12], h3f[6], h3b[6];
    Spinor<P>::load(k.in, nb[2], p2f);
    Spinor<P>::load(k.in, nb[6], p2b);
    Spinor<P>::template load_half<(F < 0)>(k.in, nb[3], h3f);
    Spinor<P>::template load_half<(B < 0)>(k.in, nb[7], h3b);
#pragma unroll
    for (int c2 = 0; c2 < 12; ++c2) acc[c2] = {(T)0, (T)0};
    staged_term_u<P, 0, F>(acc, sv, nb[0], u[0]);
    staged_term_u<P, 1, F>(acc, sv, nb[1], u[1]);
    hop_term_psi<P, 2, F>(acc, p2f, u[2]);
    hop_term_x4<P, F>(acc, h3f, u[3], sf);
    staged_term_u<P, 0, B>(acc, sv, nb[4], u[4]);
    staged_term_u<P, 1, B>(acc, sv, nb[5], u[5]);
    hop_term_psi<P, 2, B>(acc, p2b, u[6]);
    hop_term_x4<P, B>(acc, h3b, u[7], sb);
    return;
  }
#pragma unroll
  for (int c2 = 0; c2 < 12; ++c2) acc[c2] = {(T)0, (T)0};
  constexpr bool one_at_a_time = (P == WD_F64);
  staged_term<P, 0, F>(acc, k, sv, nb[0], 0, i);
  staged_term<P, 1, F>(acc, k, sv, nb[1], 1, i);
  hop_term<P, 2, F>(acc, k.in, nb[2], L, 2, i, one);
  if constexpr (one_at_a_time) __builtin_amdgcn_sched_barrier(0);
  hop_term<P, 3, F>(acc, k.in, nb[3], L, 3, i, sf);
  if constexpr (one_at_a_time) __builtin_amdgcn_sched_barrier(0);
  staged_term<P, 0, B>(acc, k, sv, nb[4], 4, i);
  staged_term<P, 1, B>(acc, k, sv, nb[5], 5, i);
  hop_term<P, 2, B>(acc, k.in, nb[6], L, 6, i, one);
  if constexpr (one_at_a_time) __builtin_amdgcn_sched_barrier(0);
  hop_term<P, 3, B>(acc, k.in, nb[7], L, 7, i, sb);
}

// One output site i of the hop with the fused epilogue
//   EPI 0: out = a H in;  1: out = X + a H in;  2: out = X - Y + a H in.
// Padding slots (vh <= i < vpad) get zeros.  Returns |stored out|^2 (FP64)
// when NORM, else 0.  PRE: links loaded up front (same arithmetic).  STG:
// x1, x2 neighbours from the block's staged input tile sv.
template <int P, bool DAG, int EPI, bool NORM, bool PRE = false, bool STG = false>
__device__ __forceinline__ double dslash_site(const KDslash &k, int i, Stage<RealOf<P>> sv = {}) {
  using T = RealOf<P>;
  double nrm = 0.0;
  if (i < k.g.vh) {
    cplx<T> acc[12];
    if constexpr (PRE) hop_all_preload<P, DAG>(k, i, acc);
    else if constexpr (STG) hop_all_staged<P, DAG>(k, i, sv, acc);
    else hop_all<P, DAG>(k, i, acc);
    const T a = (T)k.a;
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = a * acc[c];
    if constexpr (EPI >= 1) {
      cplx<T> x[12];
      Spinor<P>::load(k.X, i, x);
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[c] = acc[c] + x[c];
    }
    if constexpr (EPI == 2) {
      cplx<T> y[12];
      Spinor<P>::load(k.Y, i, y);
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[c] = acc[c] - y[c];
    }
    if (k.nt_store) Spinor<P>::template store<true>(k.out, i, acc);
    else Spinor<P>::template store<false>(k.out, i, acc);
    if constexpr (NORM) {
      // norm of what was stored (after rounding to the storage format)
      cplx<T> st[12];
      if constexpr (P == WD_F64 || P == WD_F32) {
#pragma unroll
        for (int c = 0; c < 12; ++c) st[c] = acc[c];
      } else {
        Spinor<P>::load(k.out, i, st);
      }
#pragma unroll
      for (int c = 0; c < 12; ++c) nrm += (double)st[c].re * st[c].re + (double)st[c].im * st[c].im;
    }
  } else if (i < k.g.vpad) {
    cplx<T> z[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) z[c] = {(T)0, (T)0};
    Spinor<P>::store(k.out, i, z);
  }
  return nrm;
}

}  // namespace wd
