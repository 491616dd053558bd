// Persistent multi-lattice solver: one launch covers every lattice of a batch.
//
// The lattices' half fields are cut into tiles of 64, 128 or 256 slots
// (one tile per workgroup); a work list maps each tile to its lattice.  A
// grid of (#CU x resident blocks, or a tuned number of blocks per CU)
// workgroups walks the list; each tile reads its lattice's descriptor
// (geometry, links, vector pointers, kappa, CG scalars), so lattices of any
// size share every launch.  Reductions are segmented by lattice: each tile
// stores its block partial, and a finishing kernel (one workgroup per
// lattice) sums that lattice's partials in tile order, so results do not
// depend on scheduling and no block waits on a shared counter.  A lattice
// whose CG has converged is masked: its tiles are skipped.  One pair of CG iterations over the whole batch is
// captured in a hipGraph and replayed; the host polls the per-lattice flags
// every few replays.  Outer loop: FP64 defect correction per lattice (true
// residual, solution accumulation and norms in FP64; inner CG in FP32
// arithmetic with the chosen storage precision).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "wd_blas.h"
#include "wd_hop.h"
#include "wd_solver.h"

namespace wd {

constexpr int BT = 256;  // threads of the finishing kernels; largest tile

// vector slots of a lattice
enum Slot { S_B = 0, S_X, S_R64, S_RH, S_E, S_P, S_S, S_R, S_Q, S_T, NSLOT };

struct LatDesc {
  Geom g;
  const char *links64, *links32;
  size_t lpar64, lpar32;  // link bytes per parity
  int tile0, ntiles;      // tiles per half field, first tile in the work list
  double kappa;
  char *vec[NSLOT];
  CgScalars *sc;
};

__device__ __forceinline__ size_t dev_half_bytes(int vpad, int P) {
  const size_t per = (P == WD_F64) ? 192 : (P == WD_F32) ? 96 : (P == WD_F16) ? 52 : 48;
  return per * (size_t)vpad;
}

struct Opnd {
  int slot, half;  // slot < 0: unused
};

struct KBatch {
  const LatDesc *desc;
  const int *tile_lat;
  int ntiles;           // total tiles (per half field) over the batch
  // hop
  Opnd in, out, X, Y;
  int a_mode;           // 0: a = 1; 1: a = kappa; 2: a = -kappa^2; 3: a = -kappa
  int parity;           // output parity of the hop
  int norm_field;       // double index inside CgScalars, -1: none
  int norm_accumulate;
  int j;                // CG ping-pong slot
  int nhalf;            // elementwise ops: halves per vector
  double scale;
  int use_mask;         // skip lattices whose CG is done
  double *partials;     // per work item
};

__device__ __forceinline__ char *vec_ptr(const LatDesc &d, Opnd o, int P) {
  return d.vec[o.slot] + (size_t)o.half * dev_half_bytes(d.g.vpad, P);
}

// Block partial of work item w (summed per lattice by k_batch_finish).
__device__ __forceinline__ void seg_store(double v, int w, double *partials) {
  double x[1] = {v};
  block_sum_n<1>(x);
  if (threadIdx.x == 0) partials[w] = x[0];
}

// ------------------------------------------------------------------ hop
template <int P, bool DAG, int EPI, bool NORM, int TB>
__global__ __launch_bounds__(TB) void k_batch_hop(KBatch a) {
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const int l = a.tile_lat[t];
    const LatDesc &d = a.desc[l];
    if (a.use_mask && d.sc->done) continue;
    KDslash k{};
    k.g = d.g;
    k.links = (P == WD_F64) ? d.links64 + (size_t)a.parity * d.lpar64 : d.links32 + (size_t)a.parity * d.lpar32;
    k.parity = a.parity;
    k.in = vec_ptr(d, a.in, P);
    k.out = vec_ptr(d, a.out, P);
    if constexpr (EPI >= 1) k.X = vec_ptr(d, a.X, P);
    if constexpr (EPI == 2) k.Y = vec_ptr(d, a.Y, P);
    k.a = a.a_mode == 0 ? 1.0 : a.a_mode == 1 ? d.kappa : a.a_mode == 2 ? -d.kappa * d.kappa : -d.kappa;
    k.nt_store = 1;
    const int i = (t - d.tile0) * TB + (int)threadIdx.x;
    const double nrm = dslash_site<P, DAG, EPI, NORM>(k, i);
    if constexpr (NORM) seg_store(nrm, t, a.partials);
  }
}

// ------------------------------------------------------------ elementwise
enum BOp { OP_CGU = 0, OP_PUP, OP_CONV, OP_ACC, OP_NORM };

// Work item w = h * ntiles + t covers the TS slots of tile t in half h.
template <int OP, int PA, int PB, int TS>
__global__ __launch_bounds__(TS) void k_batch_elem(KBatch a) {
  using TA = typename Spinor<PA>::real;
  using TB = typename Spinor<PB>::real;
  const int nitems_total = a.ntiles * a.nhalf;
  for (int w = blockIdx.x; w < nitems_total; w += gridDim.x) {
    const int t = w % a.ntiles, h = w / a.ntiles;
    const int l = a.tile_lat[t];
    const LatDesc &d = a.desc[l];
    CgScalars *sc = d.sc;
    if (a.use_mask && sc->done) continue;
    const int i = (t - d.tile0) * TS + (int)threadIdx.x;
    double acc = 0.0;
    if constexpr (OP == OP_CGU) {
      // X(PA) += alpha P(PB); S(PB) -= alpha Q(PB); |S|^2
      const double qq = sc->qq, rr = sc->rr[a.j];
      const bool ok = (qq > 0.0) && (qq < 1e300) && (rr < 1e300);
      if (ok && i < d.g.vh) {
        const double alpha = rr / qq;
        cplx<TA> x[12];
        cplx<TB> p[12], s[12], q[12];
        char *X = vec_ptr(d, Opnd{S_E, 0}, PA);
        Spinor<PA>::load(X, i, x);
        Spinor<PB>::load(vec_ptr(d, Opnd{S_P, 0}, PB), i, p);
        Spinor<PB>::load(vec_ptr(d, Opnd{S_S, 0}, PB), i, s);
        Spinor<PB>::load(vec_ptr(d, Opnd{S_Q, 0}, PB), i, q);
        const TA ax = (TA)alpha;
        const TB ab = (TB)alpha;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          x[c].re = fma(ax, (TA)p[c].re, x[c].re);
          x[c].im = fma(ax, (TA)p[c].im, x[c].im);
          s[c].re = fma(-ab, q[c].re, s[c].re);
          s[c].im = fma(-ab, q[c].im, s[c].im);
        }
        Spinor<PA>::store(X, i, x);
        char *S = vec_ptr(d, Opnd{S_S, 0}, PB);
        Spinor<PB>::store(S, i, s);
        if constexpr (PB != WD_F32 && PB != WD_F64) Spinor<PB>::load(S, i, s);
#pragma unroll
        for (int c = 0; c < 12; ++c) acc += (double)s[c].re * s[c].re + (double)s[c].im * s[c].im;
      }
      // every tile of the lattice stores a partial; the sum and then the
      // flags (k_batch_flags) follow in their own launches
      seg_store(acc, t, a.partials);
    } else if constexpr (OP == OP_PUP) {
      if (i < d.g.vh) {
        const TB beta = (TB)(sc->rr[1 - a.j] / sc->rr[a.j]);
        cplx<TB> r[12], p[12];
        char *Pp = vec_ptr(d, Opnd{S_P, 0}, PB);
        Spinor<PB>::load(vec_ptr(d, Opnd{S_R, 0}, PB), i, r);
        Spinor<PB>::load(Pp, i, p);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          p[c].re = fma(beta, p[c].re, r[c].re);
          p[c].im = fma(beta, p[c].im, r[c].im);
        }
        Spinor<PB>::store(Pp, i, p);
      }
    } else if constexpr (OP == OP_CONV) {
      // out(PB) = s * in(PA), s = scale (or scale / sqrt(rnorm2) if norm_field >= 0); pads zeroed
      double s = a.scale;
      if (a.norm_field >= 0) s = a.scale / sqrt(((double *)sc)[a.norm_field]);
      cplx<TB> o[12];
      if (i < d.g.vh) {
        cplx<TA> x[12];
        Spinor<PA>::load(vec_ptr(d, Opnd{a.in.slot, a.in.half + h}, PA), i, x);
#pragma unroll
        for (int c = 0; c < 12; ++c) o[c] = {(TB)(s * (double)x[c].re), (TB)(s * (double)x[c].im)};
      } else {
#pragma unroll
        for (int c = 0; c < 12; ++c) o[c] = {(TB)0, (TB)0};
      }
      if (i < d.g.vpad) Spinor<PB>::store(vec_ptr(d, Opnd{a.out.slot, a.out.half + h}, PB), i, o);
    } else if constexpr (OP == OP_ACC) {
      // X64(PB = F64) += sqrt(rnorm2) * E(PA)
      if (i < d.g.vh) {
        const double s = sqrt(sc->rnorm2);
        cplx<TA> e[12];
        cplx<double> x[12];
        Spinor<PA>::load(vec_ptr(d, Opnd{a.in.slot, h}, PA), i, e);
        char *X = vec_ptr(d, Opnd{a.out.slot, h}, WD_F64);
        Spinor<WD_F64>::load(X, i, x);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          x[c].re = fma(s, (double)e[c].re, x[c].re);
          x[c].im = fma(s, (double)e[c].im, x[c].im);
        }
        Spinor<WD_F64>::store(X, i, x);
      }
    } else {  // OP_NORM of slot `in` over nhalf halves -> sc[norm_field]
      if (i < d.g.vh) {
        cplx<TA> x[12];
        Spinor<PA>::load(vec_ptr(d, Opnd{a.in.slot, h}, PA), i, x);
#pragma unroll
        for (int c = 0; c < 12; ++c) acc += (double)x[c].re * x[c].re + (double)x[c].im * x[c].im;
      }
      seg_store(acc, w, a.partials);
    }
  }
}

// Per-lattice sums of the block partials, in work-item order (one workgroup
// per lattice).  mode 0: hop norm (items = the lattice's tiles) into
// sc[norm_field] (+= with norm_accumulate); 1: CG update, |s|^2 into ss;
// 2: norm over nhalf halves (items h * ntiles + tile) into sc[norm_field].
// Masked lattices (done) stored no partials and are left alone.
__global__ __launch_bounds__(BT) void k_batch_finish(KBatch a, int mode) {
  const int l = blockIdx.x;
  const LatDesc &d = a.desc[l];
  CgScalars *sc = d.sc;
  if (a.use_mask && sc->done) return;
  const int t0 = d.tile0, nt = d.ntiles, NT = a.ntiles;
  const int nitems = (mode == 2) ? nt * a.nhalf : nt;
  double v[1] = {0.0};
  for (int q = threadIdx.x; q < nitems; q += BT) v[0] += a.partials[(q / nt) * NT + t0 + (q % nt)];
  block_sum_n<1>(v);
  if (threadIdx.x != 0) return;
  double *dst = (mode == 1) ? &sc->ss : (double *)sc + a.norm_field;
  *dst = (mode == 0 && a.norm_accumulate) ? (*dst + v[0]) : v[0];
}

// Convergence flags after a CG update: one thread per lattice.  Breakdown
// (|M p|^2 not positive, or a non-finite scalar) ends that lattice's CG.
__global__ void k_batch_flags(const LatDesc *desc, int n, int j) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n) return;
  CgScalars *sc = desc[l].sc;
  if (sc->done) return;
  const double qq = sc->qq, rr = sc->rr[j];
  if (!(qq > 0.0) || !(qq < 1e300) || !(rr < 1e300)) {
    sc->done = 2;
    return;
  }
  sc->iters += 1;
  if (sc->ss <= sc->stop2) sc->done = 1;
  else if (sc->iters >= sc->max_iters) sc->done = 3;
}

// ============================================================ host side
struct BatchRun {
  int n = 0;
  int ntiles = 0;
  int grid = 0;
  int tb = 256;  // slots per tile = threads per workgroup
  LatDesc *d_desc = nullptr;
  int *d_tile_lat = nullptr;
  CgScalars *d_sc = nullptr;
  CgScalars *h_sc = nullptr;  // pinned
  double *partials = nullptr;
  void *vecmem = nullptr;
  std::vector<LatDesc> desc;
  hipStream_t st;
  wd_prec S;
  ~BatchRun() {
    if (d_desc) (void)hipFree(d_desc);
    if (d_tile_lat) (void)hipFree(d_tile_lat);
    if (d_sc) (void)hipFree(d_sc);
    if (h_sc) (void)hipHostFree(h_sc);
    if (partials) (void)hipFree(partials);
    if (vecmem) (void)hipFree(vecmem);
  }
};

static KBatch kb(const BatchRun &R) {
  KBatch a{};
  a.desc = R.d_desc;
  a.tile_lat = R.d_tile_lat;
  a.ntiles = R.ntiles;
  a.in = a.out = a.X = a.Y = Opnd{-1, 0};
  a.norm_field = -1;
  a.partials = R.partials;
  a.nhalf = 1;
  a.use_mask = 1;
  return a;
}

#define SC_FIELD(f) ((int)(offsetof(CgScalars, f) / sizeof(double)))

template <int P, int TB>
static void hop_launch_tb(const BatchRun &R, const KBatch &a, bool dag, int epi, bool norm) {
  dim3 g(R.grid), b(TB);
#define WD_BH(D, E, N) \
  if (dag == D && epi == E && norm == N) hipLaunchKernelGGL((k_batch_hop<P, D, E, N, TB>), g, b, 0, R.st, a);
  WD_BH(false, 0, false) WD_BH(false, 1, false) WD_BH(false, 1, true) WD_BH(false, 2, true)
  WD_BH(true, 0, false) WD_BH(true, 1, true)
#undef WD_BH
}

template <int P>
static void hop_launch(const BatchRun &R, const KBatch &a, bool dag, int epi, bool norm) {
  if (R.tb == 64) hop_launch_tb<P, 64>(R, a, dag, epi, norm);
  else if (R.tb == 128) hop_launch_tb<P, 128>(R, a, dag, epi, norm);
  else hop_launch_tb<P, 256>(R, a, dag, epi, norm);
}

static void hop_any(const BatchRun &R, wd_prec P, const KBatch &a, bool dag, int epi, bool norm) {
  switch (P) {
    case WD_F64: hop_launch<WD_F64>(R, a, dag, epi, norm); break;
    case WD_F32: hop_launch<WD_F32>(R, a, dag, epi, norm); break;
    case WD_F16: hop_launch<WD_F16>(R, a, dag, epi, norm); break;
    case WD_BF16: hop_launch<WD_BF16>(R, a, dag, epi, norm); break;
  }
  if (norm) hipLaunchKernelGGL(k_batch_finish, dim3((unsigned)R.n), dim3(BT), 0, R.st, a, 0);
}

template <int OP, int PA, int TB>
static void elem_pb_tb(const BatchRun &R, const KBatch &a, wd_prec pb) {
  dim3 g(R.grid), b(TB);
  switch (pb) {
    case WD_F64: hipLaunchKernelGGL((k_batch_elem<OP, PA, WD_F64, TB>), g, b, 0, R.st, a); break;
    case WD_F32: hipLaunchKernelGGL((k_batch_elem<OP, PA, WD_F32, TB>), g, b, 0, R.st, a); break;
    case WD_F16: hipLaunchKernelGGL((k_batch_elem<OP, PA, WD_F16, TB>), g, b, 0, R.st, a); break;
    case WD_BF16: hipLaunchKernelGGL((k_batch_elem<OP, PA, WD_BF16, TB>), g, b, 0, R.st, a); break;
  }
}

template <int OP, int PA>
static void elem_pb(const BatchRun &R, const KBatch &a, wd_prec pb) {
  if (R.tb == 64) elem_pb_tb<OP, PA, 64>(R, a, pb);
  else if (R.tb == 128) elem_pb_tb<OP, PA, 128>(R, a, pb);
  else elem_pb_tb<OP, PA, 256>(R, a, pb);
}

template <int OP>
static void elem(const BatchRun &R, const KBatch &a, wd_prec pa, wd_prec pb) {
  switch (pa) {
    case WD_F64: elem_pb<OP, WD_F64>(R, a, pb); break;
    case WD_F32: elem_pb<OP, WD_F32>(R, a, pb); break;
    case WD_F16: elem_pb<OP, WD_F16>(R, a, pb); break;
    case WD_BF16: elem_pb<OP, WD_BF16>(R, a, pb); break;
  }
  if (OP == OP_CGU || OP == OP_NORM)
    hipLaunchKernelGGL(k_batch_finish, dim3((unsigned)R.n), dim3(BT), 0, R.st, a, OP == OP_CGU ? 1 : 2);
}

// one CG iteration of every unconverged lattice (CGLS on the Schur operator)
static void batch_cg_iteration(const BatchRun &R, int j) {
  const wd_prec S = R.S;
  KBatch a = kb(R);
  // t = H_oe p ; q = p - k^2 H_eo t  (-> qq)
  a.in = {S_P, 0}; a.out = {S_T, 0}; a.parity = 1; a.a_mode = 0;
  hop_any(R, S, a, false, 0, false);
  a = kb(R);
  a.in = {S_T, 0}; a.out = {S_Q, 0}; a.X = {S_P, 0}; a.parity = 0; a.a_mode = 2; a.norm_field = SC_FIELD(qq);
  hop_any(R, S, a, false, 1, true);
  // x += alpha p ; s -= alpha q  (-> ss), then flags
  a = kb(R);
  a.j = j;
  elem<OP_CGU>(R, a, WD_F32, S);
  hipLaunchKernelGGL(k_batch_flags, dim3((R.n + 63) / 64), dim3(64), 0, R.st, (const LatDesc *)R.d_desc, R.n, j);
  // t = H^dag_oe s ; r = s - k^2 H^dag_eo t  (-> rr[1-j])
  a = kb(R);
  a.in = {S_S, 0}; a.out = {S_T, 0}; a.parity = 1; a.a_mode = 0;
  hop_any(R, S, a, true, 0, false);
  a = kb(R);
  a.in = {S_T, 0}; a.out = {S_R, 0}; a.X = {S_S, 0}; a.parity = 0; a.a_mode = 2;
  a.norm_field = SC_FIELD(rr) + (1 - j);
  hop_any(R, S, a, true, 1, true);
  // p = r + beta p
  a = kb(R);
  a.j = j;
  elem<OP_PUP>(R, a, WD_F32, S);
}

wd_status solve_batch(const wd_gauge *const *gs, int n, const void *const *b, void *const *x, const double *kappa,
                      double tol, const wd_solve_params &prm, wd_solve_info *infos) {
  auto t_start = std::chrono::steady_clock::now();
  BatchRun R;
  R.n = n;
  R.S = prm.inner_prec;
  R.tb = prm.batch_tile ? prm.batch_tile : 256;
  const wd_prec S = R.S;
  R.st = gs[0]->own_stream;
  // events: wait for every caller stream
  for (int l = 0; l < n; ++l) {
    hipEvent_t ev;
    WD_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    WD_HIP(hipEventRecord(ev, gs[l]->stream));
    WD_HIP(hipStreamWaitEvent(R.st, ev, 0));
    WD_HIP(hipEventDestroy(ev));
  }
  // descriptors and vector storage
  R.desc.resize(n);
  std::vector<int> tile_lat;
  size_t vec_bytes = 0;
  std::vector<size_t> off(n);
  for (int l = 0; l < n; ++l) {
    const Geom &G = gs[l]->geom;
    const size_t per = 2 * half_bytes(G, WD_F64) + 4 * half_bytes(G, WD_F32) + 5 * half_bytes(G, S);
    off[l] = vec_bytes;
    vec_bytes += round_up(per, 256);
    LatDesc &d = R.desc[l];
    memset(&d, 0, sizeof d);
    d.g = G;
    d.links64 = (const char *)gs[l]->links64;
    d.links32 = (const char *)gs[l]->links32;
    d.lpar64 = link_parity_bytes(G, true);
    d.lpar32 = link_parity_bytes(G, false);
    d.ntiles = G.vpad / R.tb;
    d.tile0 = (int)tile_lat.size();
    d.kappa = kappa[l];
    for (int q = 0; q < d.ntiles; ++q) tile_lat.push_back(l);
  }
  R.ntiles = (int)tile_lat.size();
  WD_HIP(hipMalloc(&R.vecmem, vec_bytes));
  WD_HIP(hipMalloc(&R.d_desc, sizeof(LatDesc) * n));
  WD_HIP(hipMalloc(&R.d_tile_lat, sizeof(int) * R.ntiles));
  WD_HIP(hipMalloc(&R.d_sc, sizeof(CgScalars) * n));
  WD_HIP(hipHostMalloc((void **)&R.h_sc, sizeof(CgScalars) * n, hipHostMallocDefault));
  WD_HIP(hipMalloc(&R.partials, sizeof(double) * 2 * R.ntiles));
  for (int l = 0; l < n; ++l) {
    LatDesc &d = R.desc[l];
    const Geom &G = d.g;
    char *c = (char *)R.vecmem + off[l];
    d.vec[S_B] = (char *)b[l];
    d.vec[S_X] = (char *)x[l];
    d.vec[S_R64] = c; c += 2 * half_bytes(G, WD_F64);
    d.vec[S_RH] = c; c += 2 * half_bytes(G, WD_F32);
    d.vec[S_E] = c; c += 2 * half_bytes(G, WD_F32);
    d.vec[S_P] = c; c += half_bytes(G, S);
    d.vec[S_S] = c; c += half_bytes(G, S);
    d.vec[S_R] = c; c += half_bytes(G, S);
    d.vec[S_Q] = c; c += half_bytes(G, S);
    d.vec[S_T] = c; c += half_bytes(G, S);
    d.sc = R.d_sc + l;
  }
  WD_HIP(hipMemcpyAsync(R.d_desc, R.desc.data(), sizeof(LatDesc) * n, hipMemcpyHostToDevice, R.st));
  WD_HIP(hipMemcpyAsync(R.d_tile_lat, tile_lat.data(), sizeof(int) * R.ntiles, hipMemcpyHostToDevice, R.st));
  // persistent grid: the resident blocks of the hop kernel on every CU, or
  // batch_blocks_per_cu blocks per CU, or (-1) one block per tile
  {
    int dev, ncu = 0, per_cu = 0;
    WD_HIP(hipGetDevice(&dev));
    WD_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const void *kern = R.tb == 64    ? (const void *)k_batch_hop<WD_F32, false, 1, true, 64>
                       : R.tb == 128 ? (const void *)k_batch_hop<WD_F32, false, 1, true, 128>
                                     : (const void *)k_batch_hop<WD_F32, false, 1, true, 256>;
    WD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, R.tb, 0));
    if (prm.batch_blocks_per_cu > 0) per_cu = prm.batch_blocks_per_cu;
    R.grid = prm.batch_blocks_per_cu < 0 ? R.ntiles : std::max(1, std::min(R.ntiles, ncu * std::max(1, per_cu)));
  }
  auto sync_sc = [&]() -> wd_status {
    WD_HIP(hipMemcpyAsync(R.h_sc, R.d_sc, sizeof(CgScalars) * n, hipMemcpyDeviceToHost, R.st));
    WD_HIP(hipStreamSynchronize(R.st));
    return WD_OK;
  };
  auto push_sc = [&]() -> wd_status {
    WD_HIP(hipMemcpyAsync(R.d_sc, R.h_sc, sizeof(CgScalars) * n, hipMemcpyHostToDevice, R.st));
    return WD_OK;
  };
  // |b|^2, x = 0, r = b
  for (int l = 0; l < n; ++l) { memset(&R.h_sc[l], 0, sizeof(CgScalars)); }
  WD_TRY(push_sc());
  {
    KBatch a = kb(R);
    a.use_mask = 0;
    a.nhalf = 2;
    a.in = {S_B, 0}; a.norm_field = SC_FIELD(bb);
    elem<OP_NORM>(R, a, WD_F64, WD_F64);
    a = kb(R); a.use_mask = 0; a.nhalf = 2;
    a.in = {S_B, 0}; a.out = {S_X, 0}; a.scale = 0.0;
    elem<OP_CONV>(R, a, WD_F64, WD_F64);
    a.out = {S_R64, 0}; a.scale = 1.0;
    elem<OP_CONV>(R, a, WD_F64, WD_F64);
    WD_HIP(hipGetLastError());
  }
  WD_TRY(sync_sc());
  std::vector<double> bb(n), rn2(n), best(n, 1e300);
  std::vector<int> active(n, 1), stalls(n, 0);
  for (int l = 0; l < n; ++l) {
    bb[l] = R.h_sc[l].bb;
    if (!(bb[l] < 1e300)) return set_error(WD_ERR_NONFINITE, "solve_batch: |b|^2 of lattice %d is not finite", l);
    rn2[l] = bb[l];
    memset(&infos[l], 0, sizeof(wd_solve_info));
  }
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (prm.use_graph) {
    WD_HIP(hipStreamBeginCapture(R.st, hipStreamCaptureModeThreadLocal));
    batch_cg_iteration(R, 0);
    batch_cg_iteration(R, 1);
    WD_HIP(hipStreamEndCapture(R.st, &graph));
    WD_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  }
  struct GraphFree {
    hipGraph_t g; hipGraphExec_t e;
    ~GraphFree() { if (e) (void)hipGraphExecDestroy(e); if (g) (void)hipGraphDestroy(g); }
  } gf{graph, exec};
  int total_iters = 0;
  const int check = std::max(2, prm.check_every & ~1);
  for (int outer = 0; outer < 200; ++outer) {
    int n_active = 0;
    for (int l = 0; l < n; ++l) {
      if (!active[l]) continue;
      if (bb[l] == 0.0 || rn2[l] <= tol * tol * bb[l] || !(rn2[l] < 1e300)) active[l] = 0;
      else if (rn2[l] < 0.5 * best[l]) { best[l] = rn2[l]; stalls[l] = 0; }
      else if (++stalls[l] >= 3) active[l] = 0;
      n_active += active[l];
    }
    if (n_active == 0 || total_iters >= prm.max_iter) break;
    // inner system set-up: rh = r / |r| (F32), s = rh_e + k H_eo rh_o (via e's odd half)
    for (int l = 0; l < n; ++l) {
      CgScalars &c = R.h_sc[l];
      const double keep_bb = c.bb;
      memset(&c, 0, sizeof c);
      c.bb = keep_bb;
      c.rnorm2 = active[l] ? rn2[l] : 1.0;
      c.stop2 = prm.inner_tol * prm.inner_tol;
      c.max_iters = std::max(1, prm.max_iter - total_iters);
      c.done = active[l] ? 0 : 1;
    }
    WD_TRY(push_sc());
    KBatch a = kb(R);
    a.nhalf = 2; a.in = {S_R64, 0}; a.out = {S_RH, 0}; a.scale = 1.0; a.norm_field = SC_FIELD(rnorm2);
    elem<OP_CONV>(R, a, WD_F64, WD_F32);
    a = kb(R);
    a.in = {S_RH, 1}; a.out = {S_E, 1}; a.X = {S_RH, 0}; a.parity = 0; a.a_mode = 1;
    hop_any(R, WD_F32, a, false, 1, false);
    a = kb(R);
    a.in = {S_E, 1}; a.out = {S_S, 0}; a.scale = 1.0;
    elem<OP_CONV>(R, a, WD_F32, S);
    // CGLS start: x = 0, r = M^dag s (-> rr[0]), p = r
    a = kb(R);
    a.in = {S_S, 0}; a.out = {S_E, 0}; a.scale = 0.0;
    elem<OP_CONV>(R, a, S, WD_F32);
    a = kb(R);
    a.in = {S_S, 0}; a.out = {S_T, 0}; a.parity = 1; a.a_mode = 0;
    hop_any(R, S, a, true, 0, false);
    a = kb(R);
    a.in = {S_T, 0}; a.out = {S_R, 0}; a.X = {S_S, 0}; a.parity = 0; a.a_mode = 2; a.norm_field = SC_FIELD(rr);
    hop_any(R, S, a, true, 1, true);
    a = kb(R);
    a.in = {S_R, 0}; a.out = {S_P, 0}; a.scale = 1.0;
    elem<OP_CONV>(R, a, S, S);
    WD_HIP(hipGetLastError());
    // CG iterations (graph replays), polling every `check` iterations
    int issued = 0;
    const int cap = std::max(1, prm.max_iter - total_iters) + 2;
    while (issued < cap) {
      for (int k = 0; k < check; k += 2) {
        if (exec) WD_HIP(hipGraphLaunch(exec, R.st));
        else { batch_cg_iteration(R, 0); batch_cg_iteration(R, 1); WD_HIP(hipGetLastError()); }
        issued += 2;
      }
      WD_TRY(sync_sc());
      bool all = true;
      for (int l = 0; l < n; ++l) all = all && R.h_sc[l].done != 0;
      if (all) break;
    }
    int it_max = 0;
    for (int l = 0; l < n; ++l) {
      if (!active[l]) continue;
      infos[l].iters += R.h_sc[l].iters;
      it_max = std::max(it_max, R.h_sc[l].iters);
    }
    total_iters += it_max;
    // e_o = rh_o + k H_oe x_e ; x += |r| e  (inactive lattices: e = 0 from zero rh)
    for (int l = 0; l < n; ++l) R.h_sc[l].done = active[l] ? 0 : 1;
    WD_TRY(push_sc());
    a = kb(R);
    a.in = {S_E, 0}; a.out = {S_E, 1}; a.X = {S_RH, 1}; a.parity = 1; a.a_mode = 1;
    hop_any(R, WD_F32, a, false, 1, false);
    a = kb(R);
    a.nhalf = 2; a.in = {S_E, 0}; a.out = {S_X, 0};
    elem<OP_ACC>(R, a, WD_F32, WD_F64);
    // r = b - D x (FP64) -> rnorm2
    for (int par = 0; par < 2; ++par) {
      a = kb(R);
      a.in = {S_X, 1 - par}; a.out = {S_R64, par}; a.X = {S_B, par}; a.Y = {S_X, par};
      a.parity = par; a.a_mode = 1; a.norm_field = SC_FIELD(rnorm2); a.norm_accumulate = par;
      hop_any(R, WD_F64, a, false, 2, true);
    }
    WD_HIP(hipGetLastError());
    WD_TRY(sync_sc());
    for (int l = 0; l < n; ++l) {
      if (!active[l]) continue;
      rn2[l] = R.h_sc[l].rnorm2;
      infos[l].outer_iters += 1;
    }
  }
  const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  wd_status worst = WD_OK;
  for (int l = 0; l < n; ++l) {
    infos[l].true_rel_resid = bb[l] > 0 ? sqrt(rn2[l] / bb[l]) : 0.0;
    infos[l].status = infos[l].true_rel_resid <= tol ? WD_OK : WD_NOT_CONVERGED;
    infos[l].seconds = sec;
    if (infos[l].status != WD_OK) worst = WD_NOT_CONVERGED;
  }
  return worst;
}

}  // namespace wd
