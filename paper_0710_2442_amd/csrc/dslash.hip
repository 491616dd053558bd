// Wilson hopping term (Eq. 3) on one checkerboard, gfx950.
//
// One lane per output site of parity p.  For each of the 8 hops the lane
// loads the neighbour spinor (structure-of-arrays, 16-byte loads), projects
// it to a half spinor with (1 +- gamma_mu), multiplies both spin rows by the
// hop's SU(3) matrix (rows 0,1 loaded, row 2 rebuilt), and adds the
// reconstructed 4-spinor.  Hop links are stored per output site (the
// backward link U^dag_{x-mu,mu} is kept at x), so all 8 link loads are
// aligned, coalesced, read-once streams; neighbour spinors are the only
// gathered, reused data.  A tuning variant stages each block's input tile in
// LDS for the x1 and x2 neighbours.  The epilogue fuses out = a*H in + X - Y
// and an FP64 |out|^2 reduction.
//
// Flop count per output site: 1320 (Sec. 5), plus 8 x 42 for rebuilding the
// third link rows.  Algorithmic bytes per output site: 8 x 12 link reals +
// 24 input reals (each input spinor is read by its 8 neighbours but counts
// once) + 24 output reals.
#include <algorithm>

#include "wd_hop.h"

namespace wd {

// EPI: 0 -> out = a H in;  1 -> out = X + a H in;  2 -> out = X - Y + a H in
// OCC > 0 asks the compiler for at least OCC waves per SIMD (fewer registers,
// possibly a few spills); OCC = 0 leaves the register budget to the compiler.
#define WD_OCC_KERNEL(OCCV, ATTR)                                                   \
  template <int P, bool DAG, int EPI, bool NORM, bool PRE>                        \
  __global__ __launch_bounds__(512) ATTR void k_dslash_o##OCCV(KDslash k) {     \
    dslash_body<P, DAG, EPI, NORM, PRE>(k);                                       \
  }

template <int P, bool DAG, int EPI, bool NORM, bool PRE>
__device__ __forceinline__ void dslash_body(const KDslash &k) {
  if (k.skip && *k.skip) return;
  double nrm;
  if (k.spl <= 1) {
    const int i = tile_of(k) * (int)blockDim.x + (int)threadIdx.x;
    nrm = dslash_site<P, DAG, EPI, NORM, PRE>(k, i);
  } else {
    // sites per lane along x4: block b covers tile s of slices spl * tg .. spl * tg + spl - 1
    const int T = k.tiles_per_slice, b = (int)blockIdx.x;
    const int s = b % T, tg = b / T;
    nrm = 0.0;
#pragma unroll 1
    for (int j = 0; j < k.spl; ++j) {
      const int i = ((tg * k.spl + j) * T + s) * (int)blockDim.x + (int)threadIdx.x;
      nrm += dslash_site<P, DAG, EPI, NORM, PRE>(k, i);
    }
  }
  if constexpr (NORM) {
    double v[1] = {nrm};
    block_sum_store<1>(v, k.partials, gridDim.x, blockIdx.x);
  }
}

WD_OCC_KERNEL(0, )
WD_OCC_KERNEL(4, __attribute__((amdgpu_waves_per_eu(4))))

// LDS staging of neighbour spinors (FP64, FP32 storage; one site per lane):
// the block first loads the input spinors of its tile's own slots and of the
// x1 rows just before and after the tile (coalesced) and stores them in LDS
// (packet-major, see Stage); then each lane takes its x1 and x2 neighbours
// from there, projecting them as it would after a memory load, and the x3 and
// x4 neighbours from memory.  The tile is k = blockDim.x / L1h whole rows of
// one x3 plane (k | L2, k >= 2) or whole planes (see dslash_stage_ok).
// Dynamic LDS: (blockDim.x + 2 L1h) spinors.
template <int P, bool DAG, int EPI, bool NORM>
__global__ __launch_bounds__(512) void k_dslash_stage(KDslash k) {
  using T = RealOf<P>;
  extern __shared__ __align__(16) char stage_lds[];
  cplx<T> *lds = (cplx<T> *)stage_lds;
  if (k.skip && *k.skip) return;
  const int n = (int)blockDim.x, t = (int)threadIdx.x, l1h = k.g.L1h;
  const int t0 = tile_of(k) * n, ns = n + 2 * l1h;
  // the rows around the tile, wrapping in its plane
  const int r0 = t0 / l1h, r1 = r0 + n / l1h - 1;  // first and last row (row = x2 + L2 (x3 + L3 x4))
  const int L2 = k.g.L[1];
  const int lo = ((r0 % L2 == 0) ? r0 + L2 - 1 : r0 - 1) * l1h;
  const int hi = ((r1 % L2 == L2 - 1) ? r1 - (L2 - 1) : r1 + 1) * l1h;
  {
    cplx<T> psi[12];
    Spinor<P>::load(k.in, t0 + t, psi);
    stage_store<T>(lds, t, ns, psi);
    if (t < 2 * l1h) {
      Spinor<P>::load(k.in, (t < l1h) ? lo + t : hi + t - l1h, psi);
      stage_store<T>(lds, n + t, ns, psi);
    }
  }
  __syncthreads();
  const double nrm =
      dslash_site<P, DAG, EPI, NORM, false, true>(k, t0 + t, Stage<T>{lds, t0, n, lo, hi, l1h, ns});
  if constexpr (NORM) {
    double v[1] = {nrm};
    block_sum_store<1>(v, k.partials, gridDim.x, blockIdx.x);
  }
}

// A block size fits LDS staging when its tile is k >= 2 whole x1 rows of one
// x3 plane (k | L2) or whole planes (L2 | k; then every x2 neighbour is in
// the tile), and the tiles cover the slots exactly.
size_t dslash_stage_lds_bytes(const Geom &G, int bs, wd_prec prec) {
  return (size_t)(bs + 2 * G.L1h) * 12 * (prec == WD_F64 ? 16 : 8);
}

bool dslash_stage_ok(const Geom &G, int bs) {
  if (bs % G.L1h) return false;
  const int rows = bs / G.L1h;
  return rows >= 2 && (G.L[1] % rows == 0 || rows % G.L[1] == 0) && G.vpad == G.vh && G.vh % bs == 0 &&
         2 * G.L1h <= bs;
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

// `lds` bytes of dynamic LDS (unused by the kernel) cap the resident blocks
// per CU (160 KiB of LDS per CU): fewer sites in flight per XCD means a
// smaller set of neighbour spinors the L2 must hold for reuse.
template <int P, bool DAG, int EPI, bool NORM>
static void launch_t(const KDslash &k, unsigned nblk, unsigned bs, unsigned lds, hipStream_t st) {
  if constexpr (P == WD_F64 || P == WD_F32) {
    if (k.stage) {
      const unsigned sb = (bs + 2 * (unsigned)k.g.L1h) * 12 * (unsigned)sizeof(cplx<RealOf<P>>);
      hipLaunchKernelGGL((k_dslash_stage<P, DAG, EPI, NORM>), dim3(nblk), dim3(bs), sb + lds, st, k);
      return;
    }
  }
  if constexpr (P != WD_F64) {
    if (k.preload) {
      if (k.occ == 4) hipLaunchKernelGGL((k_dslash_o4<P, DAG, EPI, NORM, true>), dim3(nblk), dim3(bs), lds, st, k);
      else hipLaunchKernelGGL((k_dslash_o0<P, DAG, EPI, NORM, true>), dim3(nblk), dim3(bs), lds, st, k);
      return;
    }
  }
  if (k.occ == 4) hipLaunchKernelGGL((k_dslash_o4<P, DAG, EPI, NORM, false>), dim3(nblk), dim3(bs), lds, st, k);
  else hipLaunchKernelGGL((k_dslash_o0<P, DAG, EPI, NORM, false>), dim3(nblk), dim3(bs), lds, st, k);
}

template <int P, bool DAG>
static void launch_epi(const KDslash &k, int epi, bool norm, unsigned nblk, unsigned bs, unsigned lds,
                       hipStream_t st) {
  if (norm) {
    if (epi == 0) launch_t<P, DAG, 0, true>(k, nblk, bs, lds, st);
    else if (epi == 1) launch_t<P, DAG, 1, true>(k, nblk, bs, lds, st);
    else launch_t<P, DAG, 2, true>(k, nblk, bs, lds, st);
  } else {
    if (epi == 0) launch_t<P, DAG, 0, false>(k, nblk, bs, lds, st);
    else if (epi == 1) launch_t<P, DAG, 1, false>(k, nblk, bs, lds, st);
    else launch_t<P, DAG, 2, false>(k, nblk, bs, lds, st);
  }
}

template <int P>
static void launch_prec(const KDslash &k, bool dag, int epi, bool norm, unsigned nblk, unsigned bs, unsigned lds,
                        hipStream_t st) {
  if (dag) launch_epi<P, true>(k, epi, norm, nblk, bs, lds, st);
  else launch_epi<P, false>(k, epi, norm, nblk, bs, lds, st);
}

// Largest grid of a single-RHS hop launch (smallest block size, 64).
unsigned dslash_grid_blocks(const wd_gauge *g) { return (unsigned)((g->geom.vpad + 63) / 64); }

// A variant (block size, tile order) is valid for a lattice when the block
// size divides the slots and, for groups != 0, the blocks tile the time
// slices exactly and either (G > 0) the tiles of one slice split evenly into
// G regions or (-X < 0) the slices split evenly over X lanes.
bool dslash_variant_ok(const Geom &G, int bs, int groups, int spl) {
  if (bs != 16 && bs != 64 && bs != 128 && bs != 256 && bs != 512) return false;
  if (spl != 1 && spl != 2 && spl != 4) return false;
  if (spl > 1) {
    const long slice = (long)G.vh / G.L[3];
    return groups == 0 && G.vpad == G.vh && slice % bs == 0 && G.L[3] % spl == 0;
  }
  if (groups == 0) return true;
  if (groups <= -100) {
    // box order (tile_of): nx3 boxes along x3 times 8 / nx3 along x4, whole
    // x3 planes of tiles
    const int nx3 = -groups - 100;
    if (nx3 != 1 && nx3 != 2 && nx3 != 4 && nx3 != 8) return false;
    const long plane = (long)G.L1h * G.L[1];
    return G.vpad == G.vh && plane % bs == 0 && G.L[2] % nx3 == 0 && G.L[3] % (8 / nx3) == 0;
  }
  if (groups < -16 || groups > 64) return false;
  const long slice = (long)G.vh / G.L[3];
  if (G.vpad != G.vh || slice % bs != 0) return false;
  if (groups < 0) return G.L[3] % (-groups) == 0;
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
  const int epi = a.Y ? 2 : (a.X ? 1 : 0);
  if (a.Y && !a.X) return set_error(WD_ERR_ARG, "dslash epilogue: Y given without X");
  const bool norm = a.norm_out != nullptr;
  if (norm && !k.partials) return set_error(WD_ERR_ARG, "dslash norm: no reduction buffer");
  const int pi = (int)prec;
  int bs = g->hop_block[pi], groups = g->hop_groups[pi], spl = g->hop_spl[pi];
  if (!dslash_variant_ok(g->geom, bs, groups, spl)) { bs = 256; groups = 0; spl = 1; }
  k.groups = groups;
  k.spl = spl;
  k.occ = g->hop_occ[pi];
  k.nt_store = g->hop_ntst[pi];
  k.preload = (prec != WD_F64) ? g->hop_pre[pi] : 0;
  k.stage = (prec == WD_F64 || prec == WD_F32) && spl == 1 && !k.preload && dslash_stage_ok(g->geom, bs) &&
                    dslash_stage_lds_bytes(g->geom, bs, prec) + (size_t)g->hop_lds[pi] <= (size_t)g->lds_per_block
                ? g->hop_stage[pi]
                : 0;
  k.tiles_per_slice = (groups || spl > 1) ? (int)((long)g->geom.vh / g->geom.L[3] / bs) : 0;
  const unsigned nblk = (unsigned)((g->geom.vpad + bs - 1) / bs) / (unsigned)spl;
  const unsigned lds = (unsigned)g->hop_lds[pi];
  switch (prec) {
    case WD_F64: launch_prec<WD_F64>(k, a.dagger, epi, norm, nblk, bs, lds, st); break;
    case WD_F32: launch_prec<WD_F32>(k, a.dagger, epi, norm, nblk, bs, lds, st); break;
    case WD_F16: launch_prec<WD_F16>(k, a.dagger, epi, norm, nblk, bs, lds, st); break;
    case WD_BF16: launch_prec<WD_BF16>(k, a.dagger, epi, norm, nblk, bs, lds, st); break;
    default: return set_error(WD_ERR_PREC, "dslash: unknown precision %d", (int)prec);
  }
  WD_TRY(hip_check(hipGetLastError(), "dslash launch"));
  if (norm) return launch_finish_sums(k.partials, nblk, 1, k.norm_out, 1, k.norm_accumulate, k.skip, 1, st);
  return WD_OK;
}

}  // namespace wd
