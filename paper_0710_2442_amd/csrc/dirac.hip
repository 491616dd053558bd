// Full-lattice Wilson-Dirac operator (Eq. 3 on both checkerboards) in one
// launch, so that each link is fetched from HBM once per application.
//
// A site x of parity p takes its forward links U_{x,mu} from the hop-link
// array of parity p (directions 0..3) and its backward links from the
// forward links of its neighbours x - mu, i.e. the hop-link array of parity
// 1 - p at the neighbour's index, applied as U^dag.  Those are the same bytes
// that the neighbour, processed in the same launch, reads as its own forward
// links; the block order pairs the even and odd tiles of a region on the
// same XCD so the second read is an L2 hit.  Per site the method then moves
// 4 x 12 link reals + 24 input reals + 24 output reals (96 reals: 768 B in
// FP64), against 2 x 144 reals for two single-parity launches.
//
// Epilogue as in the single-parity hop: EPI 1 out = X + a H in,
// EPI 2 out = X - Y + a H in (full fields), with an optional FP64 |out|^2.
//
// Measured on MI355X at 32^3x64 in FP64: the launch fetches ~3.5 GB, not
// 1.2 GB, because a neighbour's forward link does not stay in L2 until the
// backward hop needs it (time neighbours are a whole slice, ~19 MB of
// traffic, apart, and cached link loads also push out the spinors), so it
// runs about as fast as two tuned single-parity launches.  It is available
// through WD_ONE_PASS; the solvers keep the single-parity launches.
#include "wd_hop.h"

namespace wd {

namespace {

constexpr int DR_BS = 64;

struct KDirac {
  Geom g;
  const char *in;
  char *out;
  const char *X;
  const char *Y;
  const char *links[2];  // hop-link arrays of output parity 0 and 1
  size_t half;           // bytes per half field
  double a;
  double *norm_out;
  int norm_accumulate;
  double *partials;
  int ntiles;            // tiles of DR_BS sites per parity
};

// Block b: parity (b / 8) % 2, tile (b / 16) * 8 + b % 8.  Blocks go round
// robin to the 8 XCDs, so the even and the odd tile t of a region both run
// on XCD t % 8, as do their x3 (+-8 tiles) and x4 neighbours.
template <int P, bool DAG, int EPI, bool NORM>
__global__ __launch_bounds__(DR_BS) void k_dirac(KDirac k) {
  using T = RealOf<P>;
  const int b = (int)blockIdx.x;
  const int p = (b >> 3) & 1;
  const int tile = ((b >> 4) << 3) | (b & 7);
  const int i = tile * DR_BS + (int)threadIdx.x;
  double nrm = 0.0;
  if (tile < k.ntiles && i < k.g.vpad) {
    const size_t own = (size_t)p * k.half;
    char *out = k.out + own;
    if (i < k.g.vh) {
      const Coords c = coords_of(k.g, i, p);
      int nb[8];
      neighbours(k.g, c, i, nb);
      const T one = (T)1;
      const T sf = (c.x4 == k.g.L[3] - 1) ? (T)k.g.tbc : one;
      const T sb = (c.x4 == 0) ? (T)k.g.tbc : one;
      constexpr int F = DAG ? -1 : 1;
      constexpr int B = -F;
      const char *in = k.in + (size_t)(1 - p) * k.half;
      const char *Lo = k.links[p], *Ln = k.links[1 - p];
      cplx<T> acc[12];
#pragma unroll
      for (int q = 0; q < 12; ++q) acc[q] = {(T)0, (T)0};
      cplx<T> u[6];
      Link<T>::template load<false>(Lo, 0, i, u);
      hop_term_u<P, 0, F>(acc, in, nb[0], u, one);
      Link<T>::template load<false>(Lo, 1, i, u);
      hop_term_u<P, 1, F>(acc, in, nb[1], u, one);
      Link<T>::template load<false>(Lo, 2, i, u);
      hop_term_u<P, 2, F>(acc, in, nb[2], u, one);
      Link<T>::template load<false>(Lo, 3, i, u);
      hop_term_u<P, 3, F>(acc, in, nb[3], u, sf);
      Link<T>::template load<false>(Ln, 0, nb[4], u);
      hop_term_u<P, 0, B, true>(acc, in, nb[4], u, one);
      Link<T>::template load<false>(Ln, 1, nb[5], u);
      hop_term_u<P, 1, B, true>(acc, in, nb[5], u, one);
      Link<T>::template load<false>(Ln, 2, nb[6], u);
      hop_term_u<P, 2, B, true>(acc, in, nb[6], u, one);
      Link<T>::template load<false>(Ln, 3, nb[7], u);
      hop_term_u<P, 3, B, true>(acc, in, nb[7], u, sb);
      const T a = (T)k.a;
#pragma unroll
      for (int q = 0; q < 12; ++q) acc[q] = a * acc[q];
      if constexpr (EPI >= 1) {
        cplx<T> x[12];
        Spinor<P>::load(k.X + own, i, x);
#pragma unroll
        for (int q = 0; q < 12; ++q) acc[q] = acc[q] + x[q];
      }
      if constexpr (EPI == 2) {
        cplx<T> y[12];
        Spinor<P>::load(k.Y + own, i, y);
#pragma unroll
        for (int q = 0; q < 12; ++q) acc[q] = acc[q] - y[q];
      }
      Spinor<P>::store(out, i, acc);
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
    } else {
      cplx<T> z[12];
#pragma unroll
      for (int q = 0; q < 12; ++q) z[q] = {(T)0, (T)0};
      Spinor<P>::store(out, i, z);
    }
  }
  if constexpr (NORM) {
    double v[1] = {nrm};
    block_sum_store<1>(v, k.partials, gridDim.x, blockIdx.x);
  }
}

template <int P, bool DAG>
void launch_p(const KDirac &k, int epi, bool norm, unsigned nblk, hipStream_t st) {
#define WD_DR(E, N) \
  if (epi == E && norm == N) hipLaunchKernelGGL((k_dirac<P, DAG, E, N>), dim3(nblk), dim3(DR_BS), 0, st, k);
  WD_DR(0, false) WD_DR(1, false) WD_DR(2, false) WD_DR(0, true) WD_DR(1, true) WD_DR(2, true)
#undef WD_DR
}

}  // namespace

unsigned dirac_grid_blocks(const wd_gauge *g) {
  const unsigned nt = (unsigned)((g->geom.vpad + DR_BS - 1) / DR_BS);
  return (nt + 7) / 8 * 16;  // both parities, tiles rounded up to groups of 8
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
  k.norm_out = a.norm_out;
  k.norm_accumulate = a.norm_accumulate;
  k.partials = a.red.partials;
  k.ntiles = (int)((g->geom.vpad + DR_BS - 1) / DR_BS);
  const int epi = a.Y ? 2 : (a.X ? 1 : 0);
  const unsigned nblk = dirac_grid_blocks(g);
#define WD_DP(PR)                                          \
  if (a.dagger) launch_p<PR, true>(k, epi, norm, nblk, st); \
  else launch_p<PR, false>(k, epi, norm, nblk, st);
  switch (prec) {
    case WD_F64: WD_DP(WD_F64) break;
    case WD_F32: WD_DP(WD_F32) break;
    case WD_F16: WD_DP(WD_F16) break;
    case WD_BF16: WD_DP(WD_BF16) break;
    default: return set_error(WD_ERR_PREC, "dirac: unknown precision %d", (int)prec);
  }
#undef WD_DP
  WD_TRY(hip_check(hipGetLastError(), "dirac launch"));
  if (norm) return launch_finish_sums(k.partials, nblk, 1, k.norm_out, 1, k.norm_accumulate, nullptr, 1, st);
  return WD_OK;
}

}  // namespace wd
