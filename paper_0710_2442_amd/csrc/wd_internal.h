// Internal declarations shared by the host launchers and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/wd.h"

namespace wd {

// Lattice geometry of one handle, passed by value to kernels.
struct Geom {
  int L[4];     // L1..L4
  int L1h;      // L1 / 2
  int vh;       // V / 2 sites per parity
  int vpad;     // slots per half field
  int s2, s3, s4;  // checkerboard strides of x2, x3, x4: L1h, L1h*L2, L1h*L2*L3
  float tbc;    // time-boundary factor (+1 / -1)
};

inline size_t round_up(size_t a, size_t b) { return (a + b - 1) / b * b; }

inline Geom make_geom(const int dims[4], int tbc) {
  Geom g;
  for (int k = 0; k < 4; ++k) g.L[k] = dims[k];
  g.L1h = dims[0] / 2;
  size_t V = (size_t)dims[0] * dims[1] * dims[2] * dims[3];
  g.vh = (int)(V / 2);
  g.vpad = (int)round_up(V / 2, 256);
  g.s2 = g.L1h;
  g.s3 = g.L1h * dims[1];
  g.s4 = g.L1h * dims[1] * dims[2];
  g.tbc = (float)tbc;
  return g;
}

// Bytes per slot of one half field in each storage precision.
inline size_t slot_bytes(wd_prec p) {
  switch (p) {
    case WD_F64: return 192;
    case WD_F32: return 96;
    case WD_F16: return 52;
    case WD_BF16: return 48;
  }
  return 0;
}
inline size_t half_bytes(const Geom &g, wd_prec p) { return slot_bytes(p) * (size_t)g.vpad; }

// Hop-link arrays: for output parity p and hop d (0..3 forward along x1..x4,
// 4..7 backward), the 3x3 matrix that multiplies the projected neighbour
// (U_{x,mu} forward, U^dag_{x-mu,mu} backward) stored at the output site's
// checkerboard index as rows 0,1 -- 6 packets of 16 bytes (double) or 3
// (float) per hop.  Per parity the packets are grouped by chunks of 64 sites
// (see link_packet in wd_device.h); the two parities follow each other.
inline size_t link_parity_bytes(const Geom &g, bool dbl) { return (size_t)8 * 6 * 16 * g.vpad / (dbl ? 1 : 2); }
inline size_t link_bytes(const Geom &g, bool dbl) { return 2 * link_parity_bytes(g, dbl); }

struct Workspace;  // solver vectors and scalars (solver.hip)

}  // namespace wd

struct wd_gauge {
  wd::Geom geom;
  int dims[4];
  int tbc;
  wd_prec prec;
  int device;
  int lds_per_block;       // the device's LDS limit per block (bytes)
  int n_cu;                // compute units of the device
  int dirac_bpc[4];        // per precision: resident blocks per CU of the one-launch D_W
  int dirac_bpc_lds[2];    // FP64, FP32: the same for its LDS-staged form (0: does not fit)
  int dirac_slices[4];     // per precision: time slices per range of the one-launch D_W (0: from occupancy)
  int dirac_tile[4];       // per precision: its tiles, 2 = bricks of L1 x n2 x 2 sites, 0 = consecutive sites
  hipStream_t stream;      // caller's stream for dslash / pack
  hipStream_t own_stream;  // library stream for synchronous solves (default priority)
  void *links64;
  void *links32;
  int hop_block[4];        // per precision: block size of the single-RHS hop
  int hop_groups[4];       // per precision: XCD region groups (0 = linear order)
  int hop_occ[4];          // per precision: register-budget variant (0 or 4)
  int hop_ntst[4];         // per precision: 1 streaming output stores, 0 cached
  int mrhs_groups[4];      // per precision: block -> tile order of the multi-RHS hop
  int mrhs_block[4];       // per precision: sites per block of the FP32/16-bit multi-RHS hop
  int mrhs_rpl[4];         // per precision: right-hand sides per lane of that kernel
  int hop_lds[4];          // per precision: dynamic LDS bytes per block (caps blocks per CU)
  int hop_pre[4];          // per precision: 1 = links loaded before the first hop (not FP64)
  int hop_spl[4];          // per precision: output sites per lane along x4 (1, 2, 4)
  int hop_stage[4];        // per precision: 1 = x1/x2 neighbours from an LDS-staged tile (FP64, FP32)
  double *scratch_red;     // reduction partials / scalars for the BLAS entry points
  wd::Workspace *ws;
  void *fg_mem;            // mixed FGCR: vectors + scalars + partials, kept between solves
  size_t fg_bytes;
  double *fg_host;         // pinned scalars read back by the mixed FGCR
};

namespace wd {

// error reporting (abi.cpp)
wd_status set_error(wd_status st, const char *fmt, ...);
wd_status hip_check(hipError_t e, const char *what);

#define WD_HIP(call)                                  \
  do {                                                \
    hipError_t _e = (call);                           \
    if (_e != hipSuccess) return ::wd::hip_check(_e, #call); \
  } while (0)

#define WD_TRY(expr)                        \
  do {                                      \
    wd_status _s = (expr);                  \
    if (_s < 0) return _s;                  \
  } while (0)

// ------------------------------------------------------------ launchers
// All launchers are asynchronous on `st`.

// Eq. 3 on one checkerboard with fused epilogue:
//   out = a * H_{p,1-p} in  +  (X ? X : 0)  -  (Y ? Y : 0)
// X, Y, out are half fields of parity p; `in` is a half field of parity 1-p.
// All fields in precision `prec`; links in double for WD_F64, float otherwise.
// If norm_out != NULL the FP64 |out|^2 is written there (device).  If skip !=
// NULL and *skip != 0 the launch does nothing.
// reduction workspace needed by a grid of `nblocks` blocks summing N values
struct RedBuf {
  double *partials;   // N * nblocks block partials, summed by a finishing kernel
};

struct DslashArgs {
  const void *in = nullptr;
  void *out = nullptr;
  const void *X = nullptr;
  const void *Y = nullptr;
  double a = 1.0;
  int parity = 0;
  int dagger = 0;
  double *norm_out = nullptr;  // device
  int norm_accumulate = 0;     // add to *norm_out instead of overwriting
  const int *skip = nullptr;   // device flag
  RedBuf red{nullptr};
};
// Full-lattice D_W in one launch (dirac.hip): full fields in, out, X, Y;
// out = a H in (+ X (- Y)), optional FP64 |out|^2 over both parities.
struct DiracArgs {
  const void *in = nullptr;
  void *out = nullptr;
  const void *X = nullptr;
  const void *Y = nullptr;
  double a = 1.0;
  int dagger = 0;
  double *norm_out = nullptr;
  int norm_accumulate = 0;
  const int *skip = nullptr;  // device flag: when set, the launch does nothing
  RedBuf red{nullptr};
};
wd_status launch_dirac(const wd_gauge *g, wd_prec prec, const DiracArgs &args, hipStream_t st);
// one-launch D_W: occupancy of its kernels, queried once per handle (dirac.hip)
wd_status dirac_init(wd_gauge *g);
// whether the one-launch D_W has work items for at least half of the device's resident blocks
bool dirac_fills_device(const wd_gauge *g, wd_prec prec);
// whether (time slices per range, tile shape) is a valid one-launch D_W variant for the lattice
bool dirac_variant_ok(const wd_gauge *g, wd_prec prec, int slices, int tile);
// out[j * ostride] = (accumulate ? out[j * ostride] : 0) + sum over b of
// partials[j * nblocks + b], for j < n, in block order (one workgroup per j);
// entries whose skip[j * sstride] is set are left alone (blas.hip).
wd_status launch_finish_sums(const double *partials, unsigned nblocks, int n, double *out, int ostride,
                             int accumulate, const int *skip, int sstride, hipStream_t st);
// Time-slab decomposition (halo.hip)
size_t halo_face_bytes(const Geom &g, wd_prec prec);
wd_status launch_halo_pack(const wd_gauge *g, const void *in_slab, int nt, int face, int dagger, wd_prec prec,
                           void *face_buf, hipStream_t st);
wd_status launch_dslash_slab(const wd_gauge *g, const void *in_slab, const void *face_lo, const void *face_hi,
                             void *out_slab, double a, int parity, int t0, int nt, int dagger, wd_prec prec,
                             hipStream_t st);
unsigned dslash_grid_blocks(const wd_gauge *g);
bool dslash_variant_ok(const Geom &G, int bs, int groups, int spl = 1);
// LDS staging of the input tile fits block size bs (whole x1 rows of one plane)
bool dslash_stage_ok(const Geom &G, int bs);
// its dynamic LDS per block (FP64 or FP32 storage)
size_t dslash_stage_lds_bytes(const Geom &G, int bs, wd_prec prec);
// box order (groups -(100 + n)) of the FP32-arithmetic multi-RHS hop fits the lattice
bool mrhs_box_ok(const Geom &G, int bs, int groups);
// grid.x of the multi-RHS hop (16 sites per block)
inline size_t mrhs_grid_blocks(const wd_gauge *g) { return ((size_t)g->geom.vpad + 15) / 16; }
wd_status launch_dslash(const wd_gauge *g, wd_prec prec, const DslashArgs &args, hipStream_t st);

// multi-RHS hop: nrhs systems, right-hand side outermost.  Same epilogue as
// DslashArgs per RHS; norms go to norm_out[r * norm_stride]; RHS r is skipped
// when skip[r * skip_stride] != 0.  rhs_stride = 0 means contiguous half fields.
struct MrhsArgs {
  const void *in = nullptr;
  void *out = nullptr;
  const void *X = nullptr;
  const void *Y = nullptr;
  double a = 1.0;
  int parity = 0;
  int dagger = 0;
  int nrhs = 1;
  size_t rhs_stride = 0;
  double *norm_out = nullptr;
  int norm_stride = 1;
  int norm_accumulate = 0;
  const int *skip = nullptr;
  int skip_stride = 1;
  RedBuf red{nullptr};
};
wd_status launch_dslash_mrhs_ex(const wd_gauge *g, wd_prec prec, const MrhsArgs &a, hipStream_t st);

// multi-RHS hop (no epilogue), nrhs contiguous half fields
wd_status launch_dslash_mrhs(const wd_gauge *g, wd_prec prec, const void *in, void *out, double a,
                             int parity, int dagger, int nrhs, hipStream_t st);

// pack / unpack between canonical complex128 (device) and a field
// i.i.d. N(0,1) stored components from Philox4x64-10 (random.hip)
wd_status launch_gaussian(const wd_gauge *g, void *field, int parity, wd_prec prec, uint64_t seed, uint64_t stream,
                          hipStream_t st);
wd_status launch_pack_spinor(const wd_gauge *g, const void *canon, void *field, int parity,
                             wd_prec prec, hipStream_t st);
wd_status launch_unpack_spinor(const wd_gauge *g, const void *field, void *canon, int parity,
                               wd_prec prec, hipStream_t st);
wd_status launch_pack_gauge(const wd_gauge *g, const void *canon_dev, hipStream_t st);

}  // namespace wd
