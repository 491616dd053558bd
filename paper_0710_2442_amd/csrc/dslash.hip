// Wilson hopping term (Eq. 3) on one checkerboard, gfx950.
//
// One lane per output site of parity p.  For each of the 8 hops the lane
// loads the neighbour spinor (structure-of-arrays, 16-byte loads), projects
// it to a half spinor with (1 +- gamma_mu), multiplies both spin rows by the
// hop's SU(3) matrix (rows 0,1 loaded, row 2 rebuilt), and adds the
// reconstructed 4-spinor.  Hop links are stored per output site (the
// backward link U^dag_{x-mu,mu} is kept at x), so all 8 link loads are
// aligned, coalesced, read-once streams; neighbour spinors are the only
// gathered, reused data.  The epilogue fuses out = a*H in + X - Y and an
// FP64 |out|^2 reduction.
//
// Flop count per output site: 1320 (Sec. 5), plus 8 x 42 for rebuilding the
// third link rows.  Algorithmic bytes per output site: 8 x 12 link reals +
// 24 input reals (each input spinor is read by its 8 neighbours but counts
// once) + 24 output reals.
#include <algorithm>

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
  unsigned *counter;
  // block -> tile mapping (see tile_of)
  int groups;           // 0: linear; G > 0: G contiguous regions per time slice
  int tiles_per_slice;  // tiles (blocks) per time slice of one parity
  int occ;              // register-budget variant (0 or 4), host side only
  int nt_store;         // 1: streaming output stores; 0: cached stores
};

// Workgroups are dispatched round-robin over the XCDs (8 on MI355X), each
// with its own L2.  With `groups` = G, block b goes to region b % G and the
// blocks of one region walk its tiles slice by slice in time order, so a
// region's neighbour spinors (x1..x3 inside the slice, x4 one slice away)
// are fetched into one L2 and re-read from there.  Requires
// tiles_per_slice % G == 0 and gridDim.x == tiles_per_slice * L4.
__device__ __forceinline__ int tile_of(const KDslash &k) {
  const int b = blockIdx.x;
  if (k.groups == 0) return b;
  const int G = k.groups;
  const int per = k.tiles_per_slice / G;
  const int x = b % G, q = b / G;
  return (q / per) * k.tiles_per_slice + x * per + (q % per);
}

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

// One hop: acc += M (1 + S gamma_MU) psi_nb, M = the stored hop link.
template <int P, int MU, int S>
__device__ __forceinline__ void hop_term(cplx<RealOf<P>> (&acc)[12], const char *in, size_t vp, int nb,
                                         const char *links, int d, size_t i, RealOf<P> sign) {
  using T = RealOf<P>;
  cplx<T> psi[12];
  Spinor<P>::load(in, vp, nb, psi);
  cplx<T> h[6];
  project<MU, S>(psi, h);
  if constexpr (MU == 3) {
#pragma unroll
    for (int c = 0; c < 6; ++c) h[c] = sign * h[c];
  }
  cplx<T> u[6];
  Link<T>::load(links, d, i, u);
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
  reconstruct_add<MU, S>(acc, g);
}

template <int P, bool DAG>
__device__ __forceinline__ void hop_all(const KDslash &k, int i, cplx<RealOf<P>> (&acc)[12]) {
  using T = RealOf<P>;
  const Coords c = coords_of(k.g, i, k.parity);
  int nb[8];
  neighbours(k.g, c, i, nb);
  const size_t vp = (size_t)k.g.vpad;
  const T one = (T)1;
  const T sf = (c.x4 == k.g.L[3] - 1) ? (T)k.g.tbc : one;
  const T sb = (c.x4 == 0) ? (T)k.g.tbc : one;
  constexpr int F = DAG ? -1 : 1;  // forward hop projector (1 + F gamma)
  constexpr int B = -F;            // backward hop projector (1 + B gamma)
  const char *L = k.links;
#pragma unroll
  for (int c2 = 0; c2 < 12; ++c2) acc[c2] = {(T)0, (T)0};
  hop_term<P, 0, F>(acc, k.in, vp, nb[0], L, 0, i, one);
  hop_term<P, 1, F>(acc, k.in, vp, nb[1], L, 1, i, one);
  hop_term<P, 2, F>(acc, k.in, vp, nb[2], L, 2, i, one);
  hop_term<P, 3, F>(acc, k.in, vp, nb[3], L, 3, i, sf);
  hop_term<P, 0, B>(acc, k.in, vp, nb[4], L, 4, i, one);
  hop_term<P, 1, B>(acc, k.in, vp, nb[5], L, 5, i, one);
  hop_term<P, 2, B>(acc, k.in, vp, nb[6], L, 6, i, one);
  hop_term<P, 3, B>(acc, k.in, vp, nb[7], L, 7, i, sb);
}

// EPI: 0 -> out = a H in;  1 -> out = X + a H in;  2 -> out = X - Y + a H in
// OCC > 0 asks the compiler for at least OCC waves per SIMD (fewer registers,
// possibly a few spills); OCC = 0 leaves the register budget to the compiler.
#define WD_OCC_KERNEL(OCCV, ATTR)                                                   \
  template <int P, bool DAG, int EPI, bool NORM>                                  \
  __global__ __launch_bounds__(512) ATTR void k_dslash_o##OCCV(KDslash k) {     \
    dslash_body<P, DAG, EPI, NORM>(k);                                            \
  }

template <int P, bool DAG, int EPI, bool NORM>
__device__ __forceinline__ void dslash_body(const KDslash &k) {
  using T = RealOf<P>;
  if (k.skip && *k.skip) return;
  const int i = tile_of(k) * (int)blockDim.x + (int)threadIdx.x;
  const size_t vp = (size_t)k.g.vpad;
  double nrm = 0.0;
  if (i < k.g.vh) {
    cplx<T> acc[12];
    hop_all<P, DAG>(k, i, acc);
    const T a = (T)k.a;
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = a * acc[c];
    if constexpr (EPI >= 1) {
      cplx<T> x[12];
      Spinor<P>::load(k.X, vp, i, x);
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[c] = acc[c] + x[c];
    }
    if constexpr (EPI == 2) {
      cplx<T> y[12];
      Spinor<P>::load(k.Y, vp, i, y);
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[c] = acc[c] - y[c];
    }
    if (k.nt_store) Spinor<P>::template store<true>(k.out, vp, i, acc);
    else Spinor<P>::template store<false>(k.out, vp, i, acc);
    if constexpr (NORM) {
      // norm of what was stored (after rounding to the storage format)
      cplx<T> st[12];
      if constexpr (P == WD_F64 || P == WD_F32) {
#pragma unroll
        for (int c = 0; c < 12; ++c) st[c] = acc[c];
      } else {
        Spinor<P>::load(k.out, vp, i, st);
      }
#pragma unroll
      for (int c = 0; c < 12; ++c) nrm += (double)st[c].re * st[c].re + (double)st[c].im * st[c].im;
    }
  } else if (i < k.g.vpad) {
    cplx<T> z[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) z[c] = {(T)0, (T)0};
    Spinor<P>::store(k.out, vp, i, z);
  }
  if constexpr (NORM) {
    double v[1] = {nrm}, tot[1];
    if (grid_sum_last<1>(v, k.partials, k.counter, gridDim.x, blockIdx.x, tot)) {
      *k.norm_out = k.norm_accumulate ? (*k.norm_out + tot[0]) : tot[0];
    }
  }
}

WD_OCC_KERNEL(0, )
WD_OCC_KERNEL(4, __attribute__((amdgpu_waves_per_eu(4))))

// ---------------------------------------------------------------- mrhs
// Lanes of a wave cover 16 sites x 4 right-hand sides (lane = site + 16*rhs),
// so the four lanes of one site issue the same link addresses and the
// hardware merges them into one fetch; the waves of a block stack RHS groups
// of the same 16 sites so the links stay in L1/L2 for the whole block.
// Per-RHS epilogue as in k_dslash, per-RHS skip flags and FP64 norms.
struct KMrhs {
  KDslash k;
  int nrhs;
  size_t rhs_stride;   // bytes between right-hand sides (all operands)
  int norm_stride;     // doubles between consecutive RHS norm slots
  int skip_stride;     // ints between consecutive RHS skip flags
};

template <int P, bool DAG, int EPI, bool NORM>
__global__ __launch_bounds__(256) void k_dslash_mrhs(KMrhs m) {
  using T = RealOf<P>;
  const int lane = threadIdx.x & 15;
  const int rl = threadIdx.x >> 4;             // rhs within the block
  const int rg = blockIdx.y * 16 + rl;         // global rhs
  const int i = blockIdx.x * 16 + lane;
  const size_t vp = (size_t)m.k.g.vpad;
  const bool live = rg < m.nrhs && !(m.k.skip && m.k.skip[(size_t)rg * m.skip_stride]);
  double nrm = 0.0;
  if (live) {
    KDslash k = m.k;
    const size_t off = (size_t)rg * m.rhs_stride;
    k.in = m.k.in + off;
    char *out = m.k.out + off;
    if (i < k.g.vh) {
      cplx<T> acc[12];
      hop_all<P, DAG>(k, i, acc);
      const T a = (T)k.a;
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[c] = a * acc[c];
      if constexpr (EPI >= 1) {
        cplx<T> x[12];
        Spinor<P>::load(m.k.X + off, vp, i, x);
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = acc[c] + x[c];
      }
      if constexpr (EPI == 2) {
        cplx<T> y[12];
        Spinor<P>::load(m.k.Y + off, vp, i, y);
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = acc[c] - y[c];
      }
      Spinor<P>::store(out, vp, i, acc);
      if constexpr (NORM) {
        cplx<T> st[12];
        if constexpr (P == WD_F64 || P == WD_F32) {
#pragma unroll
          for (int c = 0; c < 12; ++c) st[c] = acc[c];
        } else {
          Spinor<P>::load(out, vp, i, st);
        }
#pragma unroll
        for (int c = 0; c < 12; ++c) nrm += (double)st[c].re * st[c].re + (double)st[c].im * st[c].im;
      }
    } else if (i < k.g.vpad) {
      cplx<T> z[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) z[c] = {(T)0, (T)0};
      Spinor<P>::store(out, vp, i, z);
    }
  }
  if constexpr (NORM) {
    // the 16 lanes of one RHS are contiguous in a wave: reduce within them
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
    const unsigned nblk = gridDim.x;
    if (lane == 0 && rg < m.nrhs)
      __hip_atomic_store(&m.k.partials[(size_t)rg * nblk + blockIdx.x], nrm, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    __shared__ int is_last;
    if (threadIdx.x == 0) {
      __threadfence();
      const unsigned ticket = atomicAdd(m.k.counter + blockIdx.y, 1u);
      is_last = (ticket == nblk - 1);
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    // last block of this RHS group: 16 lanes per RHS sum its partials in order
    double s = 0.0;
    if (rg < m.nrhs) {
      for (unsigned b = lane; b < nblk; b += 16)
        s += __hip_atomic_load(&m.k.partials[(size_t)rg * nblk + b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0 && live) {
      double *dst = m.k.norm_out + (size_t)rg * m.norm_stride;
      *dst = m.k.norm_accumulate ? (*dst + s) : s;
    }
    if (threadIdx.x == 0) __hip_atomic_store(m.k.counter + blockIdx.y, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ------------------------------------------------------------ launchers
static KDslash make_k(const wd_gauge *g, wd_prec prec, int parity) {
  KDslash k{};
  k.nt_store = 1;
  k.g = g->geom;
  const bool dbl = (prec == WD_F64);
  const char *base = (const char *)(dbl ? g->links64 : g->links32);
  k.links = base + (size_t)parity * link_parity_bytes(g->geom, dbl);
  k.parity = parity;
  return k;
}

template <int P, bool DAG, int EPI, bool NORM>
static void launch_t(const KDslash &k, unsigned nblk, unsigned bs, hipStream_t st) {
  if (k.occ == 4) hipLaunchKernelGGL((k_dslash_o4<P, DAG, EPI, NORM>), dim3(nblk), dim3(bs), 0, st, k);
  else hipLaunchKernelGGL((k_dslash_o0<P, DAG, EPI, NORM>), dim3(nblk), dim3(bs), 0, st, k);
}

template <int P, bool DAG>
static void launch_epi(const KDslash &k, int epi, bool norm, unsigned nblk, unsigned bs, hipStream_t st) {
  if (norm) {
    if (epi == 0) launch_t<P, DAG, 0, true>(k, nblk, bs, st);
    else if (epi == 1) launch_t<P, DAG, 1, true>(k, nblk, bs, st);
    else launch_t<P, DAG, 2, true>(k, nblk, bs, st);
  } else {
    if (epi == 0) launch_t<P, DAG, 0, false>(k, nblk, bs, st);
    else if (epi == 1) launch_t<P, DAG, 1, false>(k, nblk, bs, st);
    else launch_t<P, DAG, 2, false>(k, nblk, bs, st);
  }
}

template <int P>
static void launch_prec(const KDslash &k, bool dag, int epi, bool norm, unsigned nblk, unsigned bs, hipStream_t st) {
  if (dag) launch_epi<P, true>(k, epi, norm, nblk, bs, st);
  else launch_epi<P, false>(k, epi, norm, nblk, bs, st);
}

// Largest grid of a single-RHS hop launch (smallest block size, 64).
unsigned dslash_grid_blocks(const wd_gauge *g) { return (unsigned)((g->geom.vpad + 63) / 64); }

// A variant (block size, region groups) is valid for a lattice when the
// block size divides the slots and, for G > 0, the tiles of one time slice
// split evenly into G regions.
bool dslash_variant_ok(const Geom &G, int bs, int groups) {
  if (bs != 64 && bs != 128 && bs != 256 && bs != 512) return false;
  if (groups == 0) return true;
  if (groups < 0 || groups > 64) return false;
  const long slice = (long)G.vh / G.L[3];
  if (G.vpad != G.vh || slice % bs != 0) return false;
  const long tps = slice / bs;
  return tps % groups == 0;
}

wd_status launch_dslash(const wd_gauge *g, wd_prec prec, const DslashArgs &a, hipStream_t st) {
  KDslash k = make_k(g, prec, a.parity);
  k.in = (const char *)a.in;
  k.out = (char *)a.out;
  k.X = (const char *)a.X;
  k.Y = (const char *)a.Y;
  k.a = a.a;
  k.norm_out = a.norm_out;
  k.norm_accumulate = a.norm_accumulate;
  k.skip = a.skip;
  k.partials = a.red.partials;
  k.counter = a.red.counter;
  const int epi = a.Y ? 2 : (a.X ? 1 : 0);
  if (a.Y && !a.X) return set_error(WD_ERR_ARG, "dslash epilogue: Y given without X");
  const bool norm = a.norm_out != nullptr;
  if (norm && (!k.partials || !k.counter)) return set_error(WD_ERR_ARG, "dslash norm: no reduction buffer");
  const int pi = (int)prec;
  int bs = g->hop_block[pi], groups = g->hop_groups[pi];
  if (!dslash_variant_ok(g->geom, bs, groups)) { bs = 256; groups = 0; }
  k.groups = groups;
  k.occ = g->hop_occ[pi];
  k.nt_store = g->hop_ntst[pi];
  k.tiles_per_slice = groups ? (int)((long)g->geom.vh / g->geom.L[3] / bs) : 0;
  const unsigned nblk = (unsigned)((g->geom.vpad + bs - 1) / bs);
  switch (prec) {
    case WD_F64: launch_prec<WD_F64>(k, a.dagger, epi, norm, nblk, bs, st); break;
    case WD_F32: launch_prec<WD_F32>(k, a.dagger, epi, norm, nblk, bs, st); break;
    case WD_F16: launch_prec<WD_F16>(k, a.dagger, epi, norm, nblk, bs, st); break;
    case WD_BF16: launch_prec<WD_BF16>(k, a.dagger, epi, norm, nblk, bs, st); break;
    default: return set_error(WD_ERR_PREC, "dslash: unknown precision %d", (int)prec);
  }
  return hip_check(hipGetLastError(), "dslash launch");
}

template <int P, bool DAG, int EPI, bool NORM>
static void launch_mrhs_t(const KMrhs &m, dim3 grid, dim3 block, hipStream_t st) {
  hipLaunchKernelGGL((k_dslash_mrhs<P, DAG, EPI, NORM>), grid, block, 0, st, m);
}

template <int P>
static void launch_mrhs_p(const KMrhs &m, bool dag, int epi, bool norm, dim3 grid, dim3 block, hipStream_t st) {
#define WD_M(D, E, N) if (dag == D && epi == E && norm == N) launch_mrhs_t<P, D, E, N>(m, grid, block, st);
  WD_M(false, 0, false) WD_M(false, 1, false) WD_M(false, 2, false)
  WD_M(false, 0, true) WD_M(false, 1, true) WD_M(false, 2, true)
  WD_M(true, 0, false) WD_M(true, 1, false) WD_M(true, 2, false)
  WD_M(true, 0, true) WD_M(true, 1, true) WD_M(true, 2, true)
#undef WD_M
}

wd_status launch_dslash_mrhs_ex(const wd_gauge *g, wd_prec prec, const MrhsArgs &a, hipStream_t st) {
  if (a.nrhs < 1) return set_error(WD_ERR_ARG, "dslash_mrhs: nrhs = %d", a.nrhs);
  if (a.Y && !a.X) return set_error(WD_ERR_ARG, "dslash_mrhs epilogue: Y given without X");
  KMrhs m{};
  m.k = make_k(g, prec, a.parity);
  m.k.in = (const char *)a.in;
  m.k.out = (char *)a.out;
  m.k.X = (const char *)a.X;
  m.k.Y = (const char *)a.Y;
  m.k.a = a.a;
  m.k.norm_out = a.norm_out;
  m.k.norm_accumulate = a.norm_accumulate;
  m.k.skip = a.skip;
  m.k.partials = a.red.partials;
  m.k.counter = a.red.counter;
  m.nrhs = a.nrhs;
  m.rhs_stride = a.rhs_stride ? a.rhs_stride : half_bytes(g->geom, prec);
  m.norm_stride = a.norm_stride;
  m.skip_stride = a.skip_stride;
  const bool norm = a.norm_out != nullptr;
  if (norm && (!m.k.partials || !m.k.counter)) return set_error(WD_ERR_ARG, "dslash_mrhs norm: no reduction buffer");
  const int epi = a.Y ? 2 : (a.X ? 1 : 0);
  const int per_block = std::min(16, (a.nrhs + 3) / 4 * 4);
  dim3 grid((unsigned)mrhs_grid_blocks(g), (unsigned)((a.nrhs + 15) / 16));
  dim3 block((unsigned)(16 * per_block));
  switch (prec) {
    case WD_F64: launch_mrhs_p<WD_F64>(m, a.dagger, epi, norm, grid, block, st); break;
    case WD_F32: launch_mrhs_p<WD_F32>(m, a.dagger, epi, norm, grid, block, st); break;
    case WD_F16: launch_mrhs_p<WD_F16>(m, a.dagger, epi, norm, grid, block, st); break;
    case WD_BF16: launch_mrhs_p<WD_BF16>(m, a.dagger, epi, norm, grid, block, st); break;
    default: return set_error(WD_ERR_PREC, "dslash_mrhs: unknown precision %d", (int)prec);
  }
  return hip_check(hipGetLastError(), "dslash_mrhs launch");
}

wd_status launch_dslash_mrhs(const wd_gauge *g, wd_prec prec, const void *in, void *out, double a, int parity,
                             int dagger, int nrhs, hipStream_t st) {
  MrhsArgs m;
  m.in = in; m.out = out; m.a = a; m.parity = parity; m.dagger = dagger; m.nrhs = nrhs;
  return launch_dslash_mrhs_ex(g, prec, m, st);
}

}  // namespace wd
