// Multi right-hand-side Wilson hop (Eq. 3 on one checkerboard), gfx950:
// nrhs half fields share every link load.
#include <algorithm>

#include "wd_hop.h"

namespace wd {

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
  int rpl;             // right-hand sides per lane (FP32-arithmetic kernel)
  int nx3;             // > 0: box order with tile-major RHS chunks (mrhs_box)
  int nchunks;         // RHS chunks of rpl right-hand sides
  int ntiles;          // tiles of one parity
};

// Box order for the multi-RHS hop.  Dispatch lane x = b % 8 (one per XCD)
// owns one box: a contiguous 1/nx3 of the tiles of every time slice in a
// range of 8/nx3 of the slices (boxes nx3 along the slice, 8/nx3 along x4).
// The lane walks its box slice by slice, and the nchunks blocks of one tile
// (its RHS chunks) follow each other, so they run side by side on one XCD:
// the tile's links are fetched into that L2 once, and the sites in flight
// on an XCD, whose neighbours of all right-hand sides the L2 must hold, are
// fewer by the number of chunks; the next slice of the box (the time
// neighbours) is one box-slice away.  Sets the tile and the RHS chunk of
// block b.
__device__ __forceinline__ void mrhs_box(const KMrhs &m, int b, int &tile, int &chunk) {
  const int x = b & 7, q = b >> 3;
  const int T = m.k.tiles_per_slice, Tb = T / m.nx3, S = m.k.g.L[3] / (8 / m.nx3);
  const int tq = q / m.nchunks;
  chunk = q % m.nchunks;
  const int bx = x % m.nx3, bt = x / m.nx3;
  tile = (bt * S + tq / Tb) * T + bx * Tb + tq % Tb;
}

template <int P, bool DAG, int EPI, bool NORM>
__global__ __launch_bounds__(256) void k_dslash_mrhs(KMrhs m) {
  using T = RealOf<P>;
  const int lane = threadIdx.x & 15;
  const int rl = threadIdx.x >> 4;             // rhs within the block
  const int rg = blockIdx.y * 16 + rl;         // global rhs
  const int i = tile_of(m.k) * 16 + lane;
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
        Spinor<P>::load(m.k.X + off, i, x);
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = acc[c] + x[c];
      }
      if constexpr (EPI == 2) {
        cplx<T> y[12];
        Spinor<P>::load(m.k.Y + off, i, y);
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = acc[c] - y[c];
      }
      Spinor<P>::store(out, i, acc);
      if constexpr (NORM) {
        cplx<T> st[12];
        if constexpr (P == WD_F64 || P == WD_F32) {
#pragma unroll
          for (int c = 0; c < 12; ++c) st[c] = acc[c];
        } else {
          Spinor<P>::load(out, i, st);
        }
#pragma unroll
        for (int c = 0; c < 12; ++c) nrm += (double)st[c].re * st[c].re + (double)st[c].im * st[c].im;
      }
    } else if (i < k.g.vpad) {
      cplx<T> z[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) z[c] = {(T)0, (T)0};
      Spinor<P>::store(out, i, z);
    }
  }
  if constexpr (NORM) {
    // the 16 lanes of one RHS are contiguous in a wave: reduce within them;
    // the per-RHS block partials are summed by the finishing kernel
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
    if (lane == 0 && rg < m.nrhs) m.k.partials[(size_t)rg * gridDim.x + blockIdx.x] = nrm;
  }
}

// Multi-RHS hop for FP32 arithmetic (FP32, FP16 and BF16 spinors): one lane
// per output site loads its 8 hop links once into registers and then walks
// the m.rpl right-hand sides of its block's chunk (grid.y = chunk), so a link
// is read once per chunk and every spinor load of a wave is one contiguous
// run.  Chunks are dispatched one after the other (grid.x fastest), so the
// blocks resident at one time share a chunk and their neighbour spinors stay
// in L2; rpl trades that locality against link reuse and is tuned.  Per-RHS
// skip flags, epilogue and FP64 norms as in the kernel above.
constexpr int MR_CHUNK = 16;  // largest rpl

template <int P, bool DAG, int EPI, bool NORM>
__global__ __launch_bounds__(256) void k_dslash_mrhs_reg(KMrhs m) {
  using T = RealOf<P>;
  const KDslash &k = m.k;
  int tile, chunk;
  if (m.nx3 > 0) {
    mrhs_box(m, (int)blockIdx.x, tile, chunk);
  } else {
    tile = tile_of(k);
    chunk = (int)blockIdx.y;
  }
  const int i = tile * (int)blockDim.x + (int)threadIdx.x;
  const int r0 = chunk * m.rpl;
  const int r1 = min(m.nrhs, r0 + m.rpl);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __shared__ double sred[MR_CHUNK][4];
  const bool site = i < k.g.vh;
  int nb[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  cplx<T> u[8][6];
  T sf = (T)1, sb = (T)1;
  if (site) {
    const Coords c = coords_of(k.g, i, k.parity);
    neighbours(k.g, c, i, nb);
    if (c.x4 == k.g.L[3] - 1) sf = (T)k.g.tbc;
    if (c.x4 == 0) sb = (T)k.g.tbc;
#pragma unroll
    for (int d = 0; d < 8; ++d) Link<T>::load(k.links, d, i, u[d]);
  }
  const T a = (T)k.a;
  for (int r = r0; r < r1; ++r) {
    const bool live = !(k.skip && k.skip[(size_t)r * m.skip_stride]);
    double nrm = 0.0;
    if (live) {
      const size_t off = (size_t)r * m.rhs_stride;
      char *out = k.out + off;
      if (site) {
        cplx<T> acc[12];
        hop_all_u<P, DAG>(k.in + off, nb, u, sf, sb, acc);
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = a * acc[c];
        if constexpr (EPI >= 1) {
          cplx<T> x[12];
          Spinor<P>::load(k.X + off, i, x);
#pragma unroll
          for (int c = 0; c < 12; ++c) acc[c] = acc[c] + x[c];
        }
        if constexpr (EPI == 2) {
          cplx<T> y[12];
          Spinor<P>::load(k.Y + off, i, y);
#pragma unroll
          for (int c = 0; c < 12; ++c) acc[c] = acc[c] - y[c];
        }
        Spinor<P>::store(out, i, acc);
        if constexpr (NORM) {
          cplx<T> st[12];
          if constexpr (P == WD_F32) {
#pragma unroll
            for (int c = 0; c < 12; ++c) st[c] = acc[c];
          } else {
            Spinor<P>::load(out, i, st);
          }
#pragma unroll
          for (int c = 0; c < 12; ++c) nrm += (double)st[c].re * st[c].re + (double)st[c].im * st[c].im;
        }
      } else if (i < k.g.vpad) {
        cplx<T> z[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) z[c] = {(T)0, (T)0};
        Spinor<P>::store(out, i, z);
      }
    }
    if constexpr (NORM) {
      const double t = wave_sum(nrm);
      if (lane == 0) sred[r - r0][w] = t;
    }
  }
  if constexpr (NORM) {
    // per-RHS partials at partials[r * ntiles + tile], summed in tile order
    // by the finishing kernel (the same sum for every schedule)
    __syncthreads();
    if (threadIdx.x == 0) {
      const int nw = (int)blockDim.x >> 6;
      for (int r = r0; r < r1; ++r) {
        double s = 0.0;
        for (int q = 0; q < nw; ++q) s += sred[r - r0][q];
        k.partials[(size_t)r * m.ntiles + tile] = s;
      }
    }
  }
}


// ------------------------------------------------------------ launchers
static KDslash make_k_mrhs(const wd_gauge *g, wd_prec prec, int parity) {
  KDslash k{};
  k.nt_store = 1;
  k.g = g->geom;
  const bool dbl = (prec == WD_F64);
  const char *base = (const char *)(dbl ? g->links64 : g->links32);
  k.links = base + (size_t)parity * link_parity_bytes(g->geom, dbl);
  k.parity = parity;
  return k;
}

// `lds` bytes of dynamic LDS (unused by the kernel) cap the resident blocks
// per CU (160 KiB of LDS per CU): fewer sites in flight per XCD means a
// smaller set of neighbour spinors the L2 must hold for reuse.

// FP64 multi-RHS hop in box order, one right-hand side per block: block b
// is (tile, RHS) by mrhs_box with RHS chunks of one, so the nrhs blocks of a
// tile follow each other on one XCD; each runs the single-RHS hop on its RHS
// (same arithmetic, same bits), its links coming from that XCD's L2 after
// the first of them.  Norm partials per (RHS, tile) as above.
template <int P, bool DAG, int EPI, bool NORM>
__global__ __launch_bounds__(256) void k_dslash_mrhs_l2(KMrhs m) {
  int tile, r;
  mrhs_box(m, (int)blockIdx.x, tile, r);
  const bool live = !(m.k.skip && m.k.skip[(size_t)r * m.skip_stride]);
  double nrm = 0.0;
  if (live) {
    KDslash k = m.k;
    const size_t off = (size_t)r * m.rhs_stride;
    k.in = m.k.in + off;
    k.out = m.k.out + off;
    if (k.X) k.X += off;
    if (k.Y) k.Y += off;
    nrm = dslash_site<P, DAG, EPI, NORM, false>(k, tile * (int)blockDim.x + (int)threadIdx.x);
  }
  if constexpr (NORM) {
    double v[1] = {nrm};
    block_sum_n<1>(v);
    if (threadIdx.x == 0 && live) m.k.partials[(size_t)r * m.ntiles + tile] = v[0];
  }
}

template <int P, bool DAG, int EPI, bool NORM>
static void launch_mrhs_t(const KMrhs &m, dim3 grid, dim3 block, hipStream_t st) {
  if constexpr (P == WD_F64) {
    if (m.nx3 > 0) hipLaunchKernelGGL((k_dslash_mrhs_l2<P, DAG, EPI, NORM>), grid, block, 0, st, m);
    else hipLaunchKernelGGL((k_dslash_mrhs<P, DAG, EPI, NORM>), grid, block, 0, st, m);
  } else {
    hipLaunchKernelGGL((k_dslash_mrhs_reg<P, DAG, EPI, NORM>), grid, block, 0, st, m);
  }
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

// Box order of the FP32-arithmetic multi-RHS hop (groups = -(100 + nx3)):
// whole tiles per time slice, and the slices and each slice's tiles split
// evenly over the 8 boxes.
bool mrhs_box_ok(const Geom &G, int bs, int groups) {
  if (groups > -100) return false;
  const int nx3 = -groups - 100;
  if (nx3 != 1 && nx3 != 2 && nx3 != 4 && nx3 != 8) return false;
  const long slice = (long)G.vh / G.L[3];
  if (G.vpad != G.vh || slice % bs != 0) return false;
  return (slice / bs) % nx3 == 0 && G.L[3] % (8 / nx3) == 0;
}

// Block size of the multi-RHS hop: FP64 keeps 16 sites x RHS lanes, the
// others one lane per site (tunable, 64..256).
static int mrhs_block_of(const wd_gauge *g, wd_prec prec, int &groups) {
  const int pi = (int)prec;
  int bs = g->mrhs_block[pi];
  groups = g->mrhs_groups[pi];
  const bool box = mrhs_box_ok(g->geom, bs, groups);
  if (prec == WD_F64) {
    // FP64: 16-site x RHS tiles, or one RHS per block in box order
    if (box && (bs == 64 || bs == 128 || bs == 256)) return bs;
    bs = 16;
    if (groups <= -100 || !dslash_variant_ok(g->geom, bs, groups, 1)) groups = 0;
    return bs;
  }
  if (bs != 64 && bs != 128 && bs != 256) bs = 128;
  if (!box && !dslash_variant_ok(g->geom, bs, groups, 1)) groups = 0;
  return bs;
}

wd_status launch_dslash_mrhs_ex(const wd_gauge *g, wd_prec prec, const MrhsArgs &a, hipStream_t st) {
  if (a.nrhs < 1) return set_error(WD_ERR_ARG, "dslash_mrhs: nrhs = %d", a.nrhs);
  if (a.Y && !a.X) return set_error(WD_ERR_ARG, "dslash_mrhs epilogue: Y given without X");
  KMrhs m{};
  m.k = make_k_mrhs(g, prec, a.parity);
  m.k.in = (const char *)a.in;
  m.k.out = (char *)a.out;
  m.k.X = (const char *)a.X;
  m.k.Y = (const char *)a.Y;
  m.k.a = a.a;
  m.k.norm_out = a.norm_out;
  m.k.norm_accumulate = a.norm_accumulate;
  m.k.skip = a.skip;
  m.k.partials = a.red.partials;
  m.nrhs = a.nrhs;
  m.rhs_stride = a.rhs_stride ? a.rhs_stride : half_bytes(g->geom, prec);
  m.norm_stride = a.norm_stride;
  m.skip_stride = a.skip_stride;
  const bool norm = a.norm_out != nullptr;
  if (norm && !m.k.partials) return set_error(WD_ERR_ARG, "dslash_mrhs norm: no reduction buffer");
  const int epi = a.Y ? 2 : (a.X ? 1 : 0);
  int groups;
  const int bs = mrhs_block_of(g, prec, groups);
  m.k.groups = groups;
  m.k.tiles_per_slice = groups ? (int)((long)g->geom.vh / g->geom.L[3] / bs) : 0;
  dim3 grid, block;
  if (prec == WD_F64 && groups <= -100) {
    m.rpl = 1;
    m.nchunks = a.nrhs;
    m.ntiles = (int)((g->geom.vpad + bs - 1) / bs);
    m.nx3 = -groups - 100;
    grid = dim3((unsigned)(m.ntiles * m.nchunks), 1);
    block = dim3((unsigned)bs);
  } else if (prec == WD_F64) {
    const int per_block = std::min(16, (a.nrhs + 3) / 4 * 4);
    grid = dim3((unsigned)mrhs_grid_blocks(g), (unsigned)((a.nrhs + 15) / 16));
    block = dim3((unsigned)(16 * per_block));
  } else {
    m.rpl = std::max(1, std::min(MR_CHUNK, g->mrhs_rpl[(int)prec]));
    m.nchunks = (a.nrhs + m.rpl - 1) / m.rpl;
    m.ntiles = (int)((g->geom.vpad + bs - 1) / bs);
    if (groups <= -100) {
      m.nx3 = -groups - 100;
      grid = dim3((unsigned)(m.ntiles * m.nchunks), 1);
    } else {
      grid = dim3((unsigned)m.ntiles, (unsigned)m.nchunks);
    }
    block = dim3((unsigned)bs);
  }
  switch (prec) {
    case WD_F64: launch_mrhs_p<WD_F64>(m, a.dagger, epi, norm, grid, block, st); break;
    case WD_F32: launch_mrhs_p<WD_F32>(m, a.dagger, epi, norm, grid, block, st); break;
    case WD_F16: launch_mrhs_p<WD_F16>(m, a.dagger, epi, norm, grid, block, st); break;
    case WD_BF16: launch_mrhs_p<WD_BF16>(m, a.dagger, epi, norm, grid, block, st); break;
    default: return set_error(WD_ERR_PREC, "dslash_mrhs: unknown precision %d", (int)prec);
  }
  WD_TRY(hip_check(hipGetLastError(), "dslash_mrhs launch"));
  if (norm)
    return launch_finish_sums(m.k.partials, m.ntiles > 0 ? (unsigned)m.ntiles : grid.x, a.nrhs, m.k.norm_out,
                              m.norm_stride, m.k.norm_accumulate, m.k.skip, m.skip_stride, st);
  return WD_OK;
}

wd_status launch_dslash_mrhs(const wd_gauge *g, wd_prec prec, const void *in, void *out, double a, int parity,
                             int dagger, int nrhs, hipStream_t st) {
  MrhsArgs m;
  m.in = in; m.out = out; m.a = a; m.parity = parity; m.dagger = dagger; m.nrhs = nrhs;
  return launch_dslash_mrhs_ex(g, prec, m, st);
}

}  // namespace wd
