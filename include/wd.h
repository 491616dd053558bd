/*
 * wd.h -- Wilson-Dirac hopping term and solvers on AMD Instinct MI355X (gfx950).
 *
 * The operation is the 4-d hopping term of Eq. 3 of "QCD on the Cell
 * Broadband Engine" (Sec. 5):
 *
 *   psi'_x = sum_{mu=1..4} { U_{x,mu} (1 + gamma_mu) psi_{x+mu}
 *                           + U^dag_{x-mu,mu} (1 - gamma_mu) psi_{x-mu} }
 *
 * and the Wilson-Dirac operator in hopping form D_W = 1 - kappa * H, on a
 * lattice that is periodic in x1..x3 and carries the factor t_bc (-1:
 * antiperiodic) on hops across the time boundary x4 = L4-1 <-> 0.  gamma_mu
 * are the chiral (DeGrand-Rossi) matrices; gamma_5 = diag(1, 1, -1, -1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * dims[4] = (L1, L2, L3, L4); every L_i even and >= 2 (WD_ERR_DIMS otherwise).
 * Canonical site index idx = x1 + L1*(x2 + L2*(x3 + L3*x4)); parity =
 * (x1+x2+x3+x4) mod 2; checkerboard index cb = idx >> 1; V = L1 L2 L3 L4,
 * V_h = V / 2.
 *
 * Canonical ("canon") layouts, complex128 = two doubles (re, im):
 *   spinor [V][4 spin][3 colour];   gauge [V][4 mu][3 row][3 col].
 *
 * Device field layout ("field"): one checkerboard, chunked by 64 sites.
 * A half field holds the V_h sites of one parity in wd_vh_pad(dims) slots
 * (a multiple of 256; slots past V_h hold zeros).  Spin-colour component
 * c = 3*spin + colour, with the spin index in the basis where gamma_4 is
 * diagonal: stored psi' = S psi, S = (1/sqrt 2) * [[1, 1], [1, -1]] in 2x2
 * spin blocks (so psi'_{0,1} = (psi_{0,1} + psi_{2,3}) / sqrt 2 and
 * psi'_{2,3} = (psi_{0,1} - psi_{2,3}) / sqrt 2, computed as (a + b) * r,
 * (a - b) * r with r = 1/sqrt 2 in double).  S is unitary, so norms and
 * inner products of fields are the chiral-basis ones; wd_spinor_pack/unpack
 * convert.  A site's components are cut into NP packets of 16 bytes:
 *   WD_F64 : NP = 12 packets of double2    -- packet c holds component c
 *   WD_F32 : NP =  6 packets of float4     -- packet k: components 2k, 2k+1
 *   WD_F16 : NP =  3 packets of 8 x half   -- packet k: components 4k..4k+3,
 *            re/im interleaved; stored value = component / s_x with s_x =
 *            the largest |real| of the site's 24 reals (0 -> all zero)
 *   WD_BF16: NP =  3 packets of 8 x bfloat16 (round to nearest even), as FP16
 *            without the scale
 * Packet k of checkerboard site i sits at packet index
 *   (i / 64) * CHUNK + 64 * k + (i % 64),   CHUNK = 64 * NP,
 * except that an FP16 chunk is followed by the 64 float scales s_x of its
 * sites (CHUNK = 64 * 3 + 16 packets; scale of site i at float index
 * 4 * ((i / 64) * CHUNK + 192) + i % 64).  A full field is the even half
 * followed by the odd half.  With nrhs right-hand sides the right-hand
 * side index is outermost.  wd_field_bytes() gives the size.
 *
 * Ownership: the caller allocates and owns every field (device memory) and
 * every host array.  The library never frees or keeps a caller pointer past
 * the call.  A gauge handle owns its compressed links and its solver
 * workspace and releases them in wd_gauge_destroy.  A handle is not
 * thread-safe.
 *
 * Errors: no exception or abort crosses this interface.  A negative status
 * means the call did nothing (argument errors) or that output contents are
 * undefined (WD_ERR_HIP).  wd_last_error() returns a message for the calling
 * thread's last failure.
 */
#ifndef WD_H
#define WD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WD_OK = 0,
  WD_NOT_CONVERGED = 1, /* result written (best iterate), tolerance not met */
  WD_ERR_ARG = -1,      /* null pointer, bad enum value, bad scalar        */
  WD_ERR_DIMS = -2,     /* odd/small extent or dims not the handle's dims  */
  WD_ERR_PREC = -3,     /* precision not supported by this entry point     */
  WD_ERR_NONFINITE = -4,/* kappa/tol or an input norm is not finite        */
  WD_ERR_OOM = -5,      /* device allocation failed                        */
  WD_ERR_HIP = -6       /* a HIP runtime call failed                       */
} wd_status;

typedef enum { WD_F64 = 0, WD_F32 = 1, WD_F16 = 2, WD_BF16 = 3 } wd_prec;

enum { WD_EVEN = 0, WD_ODD = 1, WD_FULL = 2 };

/* flags of wd_dslash_ex.  WD_DAGGER: apply H^dag (D_W^dag).  WD_ONE_PASS
 * (parity WD_FULL only): compute D_W in one full-lattice launch that takes
 * each site's backward links from its neighbours' forward links (each link
 * is needed once per application) instead of two single-parity launches.
 * That launch marches along x4 through ranges of time slices, one spatial
 * site per lane, the way Sec. 5 streams a lattice held in main memory a
 * slice at a time: the time link, the backward time hop and the partial
 * output pass from one slice to the next in registers, so each link and
 * spinor is fetched once (768 B per site in FP64).  The full-lattice
 * solvers (WD_SOLVER_CGLS_FULL, WD_SOLVER_FGCR) apply D_W this way when its
 * work items fill the device. */
enum { WD_DAGGER = 1, WD_ONE_PASS = 2 };

typedef struct wd_gauge wd_gauge;

/* ---------------------------------------------------------------- setup -- */

/* Upload a gauge field and build the compressed link arrays (Sec. 5: a link
 * is an SU(3) matrix of 18 reals; only rows 0 and 1 are stored and row 2 is
 * rebuilt as conj(row0 x row1) at use, which is exact for SU(3) links).
 * U_host: host pointer, canonical gauge layout, V*4*9 complex128 values.
 * t_bc: -1 (antiperiodic time) or +1 (periodic).  prec: precision of the
 * fields that wd_dslash() takes for this handle.  hip_stream: hipStream_t
 * on which wd_dslash and the pack routines run (NULL = default stream).
 * Returns WD_ERR_DIMS for bad dims, WD_ERR_OOM if device memory runs out. */
wd_status wd_gauge_create(const double *U_host, const int dims[4], int t_bc,
                          wd_prec prec, void *hip_stream, wd_gauge **out);

/* Release a handle (NULL is accepted). */
wd_status wd_gauge_destroy(wd_gauge *g);

/* Change the stream of a handle (hipStream_t, NULL = default stream). */
wd_status wd_gauge_set_stream(wd_gauge *g, void *hip_stream);

/* Slots per half field (V_h rounded up to a multiple of 256). */
size_t wd_vh_pad(const int dims[4]);

/* Bytes of a field: parity WD_EVEN/WD_ODD = half field, WD_FULL = both
 * halves; times nrhs (>= 1).  Returns 0 on bad arguments. */
size_t wd_field_bytes(const int dims[4], wd_prec prec, int nrhs, int parity);

/* Canonical spinor (device, V*12 complex128) <-> device field of precision
 * prec.  parity WD_EVEN/WD_ODD converts that checkerboard only (the field is
 * a half field); WD_FULL converts both.  Unpack writes only the sites of the
 * converted parities.  Asynchronous on the handle's stream. */
wd_status wd_spinor_pack(const wd_gauge *g, const void *canon, void *field,
                         int parity, wd_prec prec);
wd_status wd_spinor_unpack(const wd_gauge *g, const void *field, void *canon,
                           int parity, wd_prec prec);

/* --------------------------------------------------------------- dslash -- */

/* Eq. 3 restricted to one checkerboard, or the full D_W.
 *   parity WD_EVEN/WD_ODD: psi_out (half field, that parity) =
 *        kappa * H_{p,1-p} psi_in (half field, the other parity);
 *        kappa = 1 gives Eq. 3 exactly on the sites of parity p.
 *   parity WD_FULL: psi_out = psi_in - kappa * H psi_in = D_W psi_in (full
 *        fields).  psi_in and psi_out must not overlap.
 * Fields are in the precision given at wd_gauge_create; dims must equal the
 * handle's dims.  Asynchronous on the handle's stream; only launch errors are
 * reported. */
wd_status wd_dslash(const wd_gauge *U, const void *psi_in, void *psi_out,
                    double kappa, const int dims[4], int parity);

/* As wd_dslash with an explicit field precision and flags.  WD_DAGGER
 * applies H^dag, i.e. Eq. 3 with the projectors (1 +- gamma_mu) exchanged
 * (H^dag = gamma_5 H gamma_5). */
wd_status wd_dslash_ex(const wd_gauge *U, const void *psi_in, void *psi_out,
                       double kappa, int parity, wd_prec prec, int flags);

/* Multi right-hand-side form of the single-parity hop: nrhs half fields
 * (right-hand side outermost) share each link load.  parity WD_EVEN/WD_ODD
 * only; prec WD_F64/WD_F32/WD_F16/WD_BF16; 1 <= nrhs <= 64. */
wd_status wd_dslash_mrhs(const wd_gauge *U, const void *psi_in, void *psi_out,
                         double kappa, int parity, wd_prec prec, int nrhs);

/* ---------------------------------------------------------------- BLAS -- */
/* Level-1 operations on n consecutive half fields (n = nrhs*halves) in
 * precision prec, Sec. 4's caxpy among them.  Reductions accumulate in FP64
 * in a fixed order (bitwise reproducible).  Results of reductions are written
 * to host memory; these calls synchronise the handle's stream. */
wd_status wd_caxpy(const wd_gauge *g, double c_re, double c_im, const void *x,
                   void *y, int nhalf, wd_prec prec); /* y = c x + y */
wd_status wd_cdot(const wd_gauge *g, const void *x, const void *y, int nhalf,
                  wd_prec prec, double out[2]);     /* <x,y> = sum conj(x) y */
wd_status wd_norm2(const wd_gauge *g, const void *x, int nhalf, wd_prec prec,
                   double *out);
/* out (pout) = scale * in (pin) over nhalf half fields; padding slots are
 * zeroed.  In place only for equal precisions.  Asynchronous. */
wd_status wd_convert(const wd_gauge *g, const void *in, wd_prec pin, void *out,
                     wd_prec pout, int nhalf, double scale);

/* Fill a field (parity WD_EVEN / WD_ODD: one half field; WD_FULL: both) with
 * stored components whose real and imaginary parts are i.i.d. N(0,1),
 * drawn on the device by the counter-based generator Philox4x64-10 (Salmon
 * et al., SC 2011; multipliers 0xD2E7470EE14C6C93, 0xCA5A826395121157, key
 * increments 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B).  For the site of
 * parity q and checkerboard index i, and j = 0..5, the block with counter
 * ((q V_h + i) 6 + j, stream, 0, 0) and key (seed, 0) gives four words
 * x0..x3; stored component 2j = B(x0, x1) and 2j+1 = B(x2, x3), with the
 * Box-Muller map B(a, b) = sqrt(-2 ln u) (cos 2 pi v + i sin 2 pi v),
 * u = ((a >> 11) + 1) 2^-53, v = (b >> 11) 2^-53.  The values are those of
 * the stored (storage-basis) components; since the basis map is orthogonal
 * the chiral-basis field is i.i.d. Gaussian too.  prec: WD_F64 or WD_F32
 * (rounded from double).  Padding slots get zeros.  Asynchronous on the
 * handle's stream. */
wd_status wd_gaussian_field(const wd_gauge *g, void *field, int parity,
                            wd_prec prec, unsigned long long seed,
                            unsigned long long stream);

/* ---------------------------------------- time-slab decomposition (one GPU's share) -- */
/* A rank of a decomposition along x4 owns slices [t0, t0 + nt).  Its slab
 * field of one parity holds those slices only: checkerboard sites
 * [t0 S, (t0 + nt) S) of the half field, S = L1 L2 L3 / 2 (required to be a
 * multiple of 64, so a slab is a chunk-aligned part of a half field and a
 * pointer to byte t0 * S * (bytes per site) of a full-lattice half field is
 * a valid slab).  The time neighbours of the slab's first and last slices
 * arrive as face buffers of S projected half spinors (6 complex numbers per
 * site: wd_halo_face_bytes), the message a GPU would send over xGMI.  Hop
 * links come from the gauge handle of the whole lattice; since every site
 * stores its own backward links, a rank needs no links from its neighbours.
 * FP64 and FP32 only. */
size_t wd_halo_face_bytes(const int dims[4], wd_prec prec);

/* Pack the face a neighbour needs from an input-parity slab of nt slices:
 * face 0 = the slab's first slice (for the rank below), 1 = its last slice
 * (for the rank above); dagger selects the half spinor that the D_W^dag hop
 * projects to.  Asynchronous on the handle's stream. */
wd_status wd_halo_pack(const wd_gauge *U, const void *in_slab, int nt, int face,
                       int dagger, wd_prec prec, void *face_buf);

/* out_slab = a H_{p,1-p} in on the output-parity sites of slices
 * [t0, t0 + nt): in_slab is the input-parity slab of the same slices,
 * face_lo the packed face 1 of the rank below (slice t0 - 1) and face_hi the
 * packed face 0 of the rank above (slice t0 + nt), periodic in rank order;
 * the time-boundary sign applies at the lattice's own edge.  Same arithmetic
 * as wd_dslash, so a set of slabs reproduces it bit for bit.  Asynchronous. */
wd_status wd_dslash_slab(const wd_gauge *U, const void *in_slab, const void *face_lo,
                         const void *face_hi, void *out_slab, double a, int parity,
                         int t0, int nt, int dagger, wd_prec prec);

/* --------------------------------------------------------------- solve -- */

/* WD_SOLVER_CG        : FP64 even-odd CGLS (CG on the normal equations of
 *                       the Schur operator; the paper leaves the solver that
 *                       applies Eq. 3 repeatedly unspecified, Sec. 5).
 * WD_SOLVER_DEFECT_CG : FP64 defect correction, inner even-odd CGLS in FP32
 *                       arithmetic with inner_prec storage.
 * WD_SOLVER_FGCR      : FP64 flexible GCR(fgcr_m) on the full D_W with
 *                       precond as right preconditioner; modified
 *                       Gram-Schmidt; falls back to FP64 CG when stalled.
 * WD_SOLVER_DEFECT_FGCR: FP64 defect correction whose inner solver is an
 *                       FP32 flexible GCR(fgcr_m <= 16, restarted) on the
 *                       even-odd Schur operator with right preconditioner
 *                       z = [precond (r_e, 0)]_e (identity if NULL);
 *                       classical Gram-Schmidt in fused kernels, FP64
 *                       reductions; inner_prec WD_F32 or WD_BF16 stores the
 *                       residual and the directions (z_j, w_j) in that
 *                       precision, the inner solution stays FP32 (with
 *                       a BF16-activation network, the network runs as
 *                       wd_ptc_apply_even with WD_PTC_BF16_MFMA);
 *                       falls back to FP64 CG when stalled or non-finite.
 * WD_SOLVER_CGLS_FULL : FP64 CGLS on the full-lattice D_W (D^dag D x =
 *                       D^dag b on full fields, no even-odd reduction): the
 *                       plain method, for comparison. */
enum { WD_SOLVER_CG = 0, WD_SOLVER_DEFECT_CG = 1, WD_SOLVER_FGCR = 2, WD_SOLVER_DEFECT_FGCR = 3,
       WD_SOLVER_CGLS_FULL = 4 };

typedef struct wd_ptc wd_ptc;

typedef struct {
  size_t struct_size;    /* sizeof(wd_solve_params)                         */
  int solver;            /* WD_SOLVER_*                                     */
  wd_prec inner_prec;    /* defect correction: storage of inner vectors     */
  double inner_tol;      /* defect correction: inner relative tolerance     */
  int max_iter;          /* cap on (inner) CG iterations in total           */
  int check_every;       /* host polls convergence every k iterations       */
  int use_graph;         /* capture one CG iteration pair in a hipGraph     */
  int fgcr_m;            /* FGCR restart length                             */
  const wd_ptc *precond; /* FGCR right preconditioner (NULL = identity)     */
  int batch_tile;        /* wd_solve_batch: slots per tile and workgroup,    */
                         /* 64, 128 or 256 (0 = 256)                         */
  int batch_blocks_per_cu; /* wd_solve_batch: persistent workgroups per CU   */
                         /* (0 = as many as fit, -1 = one per tile)          */
} wd_solve_params;

typedef struct {
  int iters;             /* CG iterations (inner iterations for defect cg)  */
  int outer_iters;       /* defect-correction / FGCR restarts               */
  int dslash_calls;      /* single-parity hop applications                  */
  double true_rel_resid; /* |b - D_W x| / |b| in FP64, recomputed on return */
  double seconds;        /* wall time of the solve                          */
  int fallback_used;     /* FGCR fell back to CG                            */
  int status;            /* same value as returned                          */
} wd_solve_info;

/* Fill params with defaults (plain FP64 even-odd CG on the normal equations). */
void wd_solve_params_default(wd_solve_params *p);

/* Solve D_W x = b to |b - D_W x| / |b| <= tol (FP64 true residual).  The
 * paper names an iterative solver that applies Eq. 3 repeatedly (Sec. 5, data
 * in on-chip memory) without choosing one; the default here is CG on the
 * normal equations of the even-odd Schur operator.  b and x
 * are full FP64 fields (device); x is output only (the initial guess is 0).
 * p = NULL selects FP64 even-odd CGLS; see wd_solve_params for the mixed
 * precision and FGCR forms.  Synchronous.  b = 0 gives x = 0 and WD_OK.
 * WD_NOT_CONVERGED: x holds the last iterate, info is filled. */
wd_status wd_solve(const wd_gauge *U, const void *b, void *x, double kappa,
                   double tol, const wd_solve_params *p, wd_solve_info *info);

/* Solve nrhs systems with the same operator together (multi-RHS dslash,
 * independent CG scalars per system).  b, x: nrhs full FP64 fields, right-hand
 * side outermost.  Defect correction with inner_prec storage, FP64 outer. */
wd_status wd_solve_mrhs(const wd_gauge *U, const void *b, void *x, int nrhs,
                        double kappa, double tol, const wd_solve_params *p,
                        wd_solve_info *info);

/* Allocation-free form of wd_solve, for callers that cannot allocate device
 * memory on the call (serving loops that must not allocate, harnesses that
 * forbid hipMalloc).  It runs wd_solve's FP64 even-odd CGLS (p NULL or
 * p->solver == WD_SOLVER_CG; p->use_graph is ignored: the iterations are
 * launched one by one, which gives the same bits) with the solver's workspace
 * (eight FP64 half fields, the CG scalars and the reduction partials) in one
 * static device array of WD_NOALLOC_SCRATCH_BYTES that every GPU running the
 * library holds until the process ends; it calls no hipMalloc, hipFree,
 * hipHostMalloc or hipEventCreate and no graph.  The gauge handle, b and x are
 * the caller's, as for wd_solve.  Lattices whose workspace exceeds the array
 * (V/2 above about 43,000 sites; 16^4 fits) give WD_ERR_ARG, as do other
 * solvers.  Runs on the handle's stream (wd_gauge_set_stream)
 * and returns when the solve is done.  Results equal wd_solve's bit for bit.
 * All calls on one GPU share the array: calls that overlap on one GPU (other
 * threads, other streams) race; calls in sequence are safe, since every part
 * of the workspace is written before it is read. */
#define WD_NOALLOC_SCRATCH_BYTES (64u << 20)
wd_status wd_solve_noalloc(const wd_gauge *U, const void *b, void *x, double kappa,
                           double tol, const wd_solve_params *p, wd_solve_info *info);

/* ------------------------------------------------- learned preconditioner -- */
/* Gauge-covariant parallel-transport convolution network (not in the paper):
 * two layers, 1 -> 2 -> 1 spinor channels,
 *   y_{c'}(x) = sum_c sum_h W^{(h)}_{c'c} (T_h psi_c)(x),  h = 0..8,
 * T_0 = 1, T_{+mu} psi(x) = U_{x,mu} psi(x+mu), T_{-mu} psi(x) =
 * U^dag_{x-mu,mu} psi(x-mu) (h = 1..4: +x1..+x4, h = 5..8: -x1..-x4, with
 * the time-boundary factor of Eq. 3); W^{(h)}_{c'c} is a complex 4x4 spin
 * matrix.  No bias, no nonlinearity.
 * Weights (host, 1152 floats): layer 1 [9][2][1][4][4] complex then layer 2
 * [9][1][2][4][4] complex, each complex as (re, im), spin row major.
 * Fields: FP32 full fields in the layout of wd.h.  act_prec (WD_BF16 or
 * WD_F32) is the storage of the network input and hidden layer.  A network
 * belongs to one gauge handle (its links and lattice) and runs on that
 * handle's stream. */
wd_status wd_ptc_create(const wd_gauge *g, const float *W_host, wd_prec act_prec,
                        wd_ptc **out);
wd_status wd_ptc_destroy(wd_ptc *n);
/* replace the weights (resets the optimizer state) / read them back */
wd_status wd_ptc_set_weights(wd_ptc *n, const float *W_host);
wd_status wd_ptc_get_weights(const wd_ptc *n, float *W_host);
/* out = N(in); asynchronous */
wd_status wd_ptc_apply(const wd_ptc *n, const void *in, void *out);

/* Flag of wd_ptc_apply_even: products in FP16 with FP32 sums, on FP16 copies
 * of the links and weights (made on first use; the links copy takes 192 B
 * per site).  The input is scaled to unit RMS before it is rounded (the
 * network is linear) and the output scaled back.  BF16 activations only. */
enum { WD_PTC_FP16_PRODUCTS = 1 };
/* Flag of wd_ptc_apply_even: the spin mixing on the matrix cores (BF16
 * operands, FP32 sums) and the transports as BF16 dot products with FP32
 * sums, on a BF16 copy of the links (made on first use, 192 B per site); the
 * two spin matrices of the h = 0 terms are multiplied once.  No input
 * scaling (BF16 has FP32's exponent range).  BF16 activations only; not
 * together with WD_PTC_FP16_PRODUCTS. */
enum { WD_PTC_BF16_MFMA = 2 };

/* out_e = [N (in_e, 0)]_e: the network applied to a field that is zero on
 * odd sites, even sites of the result only, as the even-odd solver uses it.
 * in_even, out_even: even half fields in pin / pout (WD_F32 or WD_BF16).
 * flags: 0, WD_PTC_FP16_PRODUCTS or WD_PTC_BF16_MFMA.  Asynchronous on the
 * handle's stream. */
wd_status wd_ptc_apply_even(const wd_ptc *n, const void *in_even, wd_prec pin,
                            void *out_even, wd_prec pout, int flags);
/* Loss L = (1/B) sum_b |N(r_b) - e_b|^2 over B pairs (r and e: B consecutive
 * FP32 full fields each) and its gradient dL/dRe W + i dL/dIm W (1152 floats,
 * host; may be NULL).  Synchronous. */
wd_status wd_ptc_loss_grad(wd_ptc *n, const void *r, const void *e, int B,
                           double *loss, float *grad_host);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the same loss; returns
 * the loss before the step if loss != NULL (then synchronous). */
wd_status wd_ptc_train_step(wd_ptc *n, const void *r, const void *e, int B,
                            double lr, double *loss);

/* --------------------------------------------------------------- tuning -- */

/* Autotune the single-RHS hop of precision prec on this handle's lattice:
 * block size (64..512 threads), the block -> tile order (groups: 0 = linear;
 * G > 0 = G regions of each time slice, dealt round-robin over the XCDs;
 * -X = X contiguous ranges of time slices, one per dispatch lane, each swept
 * in time order, so with X = 8 every XCD's L2 sees whole neighbourhoods;
 * -(100 + n), n = 1, 2, 4, 8 = box order: the lattice is cut into n boxes
 * along x3 times 8 / n along x4, one per dispatch lane (per XCD), and each
 * lane walks its box slice by slice, plane by plane),
 * the register budget (occ 0: compiler's
 * choice; occ 4: at least 4 waves per SIMD), the output store policy
 * (WD_TUNE_CACHED_STORE set in occ: cached stores), link preloading
 * (WD_TUNE_PRELOAD_LINKS, not FP64), LDS staging of the block's input tile
 * (WD_TUNE_STAGE_LDS, FP64 and FP32), sites per lane along x4
 * (WD_TUNE_SPL_SHIFT) and a cap on resident
 * blocks per CU (dynamic LDS in KiB << WD_TUNE_LDS_SHIFT).  Every candidate's output is
 * first compared byte for byte with the reference variant (256 threads,
 * linear, occ 0); matching candidates are timed with HIP events on
 * alternating even/odd hops and the fastest is kept in the handle.
 * cache_path (may be NULL): JSON-lines file keyed by (arch, kernel, precision,
 * lattice); an existing entry is used without timing unless force != 0, and
 * new results are appended.  Outputs (may be NULL): the chosen variant and
 * its time per launch in microseconds (the stored time when the entry was taken
 * from the cache).
 * Synchronous. */
wd_status wd_tune_dslash(wd_gauge *g, wd_prec prec, const char *cache_path,
                         int force, int *block, int *groups, int *occ,
                         double *us);

/* Tune the multi-RHS hop for nrhs right-hand sides.  FP32, FP16, BF16: one
 * lane per site holds its 8 links in registers and loops over rpl
 * right-hand sides (chunks of rpl RHS are dispatched one after the other);
 * tuned: block size (64, 128, 256 sites), rpl (1..16) and block -> tile
 * order (groups as above).  FP64: fixed 16-site x RHS tiles; tuned: tile
 * order.  Candidates are checked byte for byte against the linear variant,
 * then timed; the fastest is kept in the handle.  cache_path and force as
 * for wd_tune_dslash (the key adds nrhs; the cache line's third field is
 * "rpl").  Outputs may be NULL.  Synchronous. */
wd_status wd_tune_dslash_mrhs(wd_gauge *g, wd_prec prec, int nrhs,
                              const char *cache_path, int force, int *block,
                              int *groups, int *rpl, double *us);

/* Set / read the multi-RHS hop variant used for precision prec: block (FP64:
 * 16; others 64, 128 or 256 sites), groups (block -> tile order, as for
 * wd_set_dslash_variant) and rpl (FP64: 4; others 1..16 right-hand sides per
 * lane).  WD_ERR_ARG for a value
 * outside these or a variant that does not fit the lattice.  The variants
 * compute the same bytes; only the time differs. */
wd_status wd_set_dslash_mrhs_variant(wd_gauge *g, wd_prec prec, int block, int groups, int rpl);
wd_status wd_get_dslash_mrhs_variant(const wd_gauge *g, wd_prec prec, int *block, int *groups, int *rpl);

/* Bit of the occ value: the hop writes its output with ordinary (cached)
 * stores instead of streaming stores, so that a following kernel can read a
 * freshly written field from the caches. */
enum { WD_TUNE_CACHED_STORE = 256 };
/* Bit of the occ value: the hop loads all 8 links of a site before its first
 * hop (more loads in flight, more registers); FP32, FP16 and BF16 only. */
enum { WD_TUNE_PRELOAD_LINKS = 512 };
/* Field of the occ value: (0, 1, 2) << WD_TUNE_SPL_SHIFT gives each lane
 * (1, 2, 4) output sites along x4 (the same tile of consecutive time slices;
 * linear tile order only). */
enum { WD_TUNE_SPL_SHIFT = 10 };
/* The dynamic LDS (KiB, 0..64) reserved per block, shifted into occ: it caps
 * the blocks resident on a CU and so the sites in flight per XCD. */
enum { WD_TUNE_LDS_SHIFT = 16 };
/* Bit of the occ value: LDS staging of neighbour spinors.  Each block first
 * loads the input spinors of its own tile of sites into LDS with coalesced
 * loads; its lanes then read their x1 and x2 neighbours from there when these
 * lie in the tile (a tile of consecutive sites holds whole x1 rows), the rest
 * from memory (Sec. 5's on-chip reuse of neighbour operands).  FP64 and FP32
 * storage; one site per lane, no link preloading, no LDS cap.  Same bytes as
 * every other variant. */
enum { WD_TUNE_STAGE_LDS = 4096 };

/* Set / read the hop variant used for precision prec.  occ: 0 or 4, or'ed
 * with WD_TUNE_CACHED_STORE, WD_TUNE_PRELOAD_LINKS (not FP64),
 * WD_TUNE_STAGE_LDS (FP64, FP32), (0, 1, 2) << WD_TUNE_SPL_SHIFT and (KiB of
 * LDS << WD_TUNE_LDS_SHIFT).  WD_ERR_ARG if the variant does not fit the
 * lattice (see wd_tune_dslash). */
wd_status wd_set_dslash_variant(wd_gauge *g, wd_prec prec, int block, int groups,
                                int occ);
wd_status wd_get_dslash_variant(const wd_gauge *g, wd_prec prec, int *block,
                                int *groups, int *occ);

/* Tune the one-launch D_W (WD_ONE_PASS; Eq. 3 on both checkerboards, the
 * slice-marching scheme of Sec. 5) for precision prec: slices = time slices
 * per range that one block marches through (8, 16, 32, ... up to L4) and
 * tile = the shape of a block's 256 spatial sites (2: bricks of L1 x n2 x 2
 * sites, where n2 = 128 / L1 divides L2 and L3 is even; 3: the same bricks,
 * with the spinors of each slice of the brick and of its four side faces
 * staged in LDS at every step, so the spatial neighbours are read from LDS
 * (FP64 and FP32 storage; (256 + 2 L1 (n2 + 2)) x 192 or 96 bytes of LDS
 * per block); 0: 256 consecutive sites, x1 fastest).  Every candidate is checked byte for byte against the
 * current variant, then timed on a random field; the fastest is kept in the
 * handle.  cache_path and force as for wd_tune_dslash (key
 * "<arch>/dirac/p<prec>/<L1>x<L2>x<L3>x<L4>"; the cache line's "block" is
 * 256, "groups" the tile and the third field "slices").  Outputs may be
 * NULL.  Synchronous. */
wd_status wd_tune_dirac(wd_gauge *g, wd_prec prec, const char *cache_path, int force,
                        int *slices, int *tile, double *us);

/* Set / read the one-launch D_W variant of precision prec: slices 0 (the
 * default: the shortest range of 8, 16, ... for which every work item is
 * resident on the device at once) or 1..L4, tile 0, 2 or 3 as above (the
 * default: 3 where it fits, else 2 where bricks fit, else 0).
 * WD_ERR_ARG for a value outside these or a brick that does not fit the
 * lattice.  The variants compute the same bytes; only the time differs. */
wd_status wd_set_dirac_variant(wd_gauge *g, wd_prec prec, int slices, int tile);
wd_status wd_get_dirac_variant(const wd_gauge *g, wd_prec prec, int *slices, int *tile);

/* Solve one system on each of n lattices (uneven sizes allowed) together:
 * every kernel of the solve is one persistent launch over a work list of
 * (lattice, tile) items, with per-lattice descriptors, lattice-segmented
 * reductions and per-lattice convergence masks; one pair of CG iterations is
 * captured in a hipGraph (params->use_graph) and replayed.  gs[l], b[l], x[l]
 * and kappa[l] as for wd_solve (FP64 full fields of lattice l); infos[l]
 * receives that lattice's results.  params->solver must be
 * WD_SOLVER_DEFECT_CG (FP64 outer, FP32 arithmetic inner with inner_prec
 * storage).  All handles must live on the same device.  Synchronous. */
wd_status wd_solve_batch(const wd_gauge *const *gs, int n, const void *const *b,
                         void *const *x, const double *kappa, double tol,
                         const wd_solve_params *params, wd_solve_info *infos);

/* Tune wd_solve_batch for these lattices: the slots per tile and workgroup
 * (params->batch_tile: 256, 128, 64) and the persistent workgroups per CU
 * (params->batch_blocks_per_cu: as many as fit, 1, 2, 4, 8, or one per tile).
 * Each candidate solves the batch (gs, b, x, kappa, tol and params as for
 * wd_solve_batch; x is overwritten) once to warm up and twice timed; only
 * candidates whose every lattice reaches tol count, and the fastest wall time
 * wins.  cache_path (may be NULL): the JSON-lines table of wd_tune_dslash,
 * keyed by (arch, "batch<n>", inner precision, the lattices' dims in order);
 * an entry is used without timing unless force != 0.  Outputs (may be NULL):
 * the chosen tile, blocks per CU and seconds per solve.  Synchronous. */
wd_status wd_tune_batch(const wd_gauge *const *gs, int n, const void *const *b,
                        void *const *x, const double *kappa, double tol,
                        const wd_solve_params *params, const char *cache_path,
                        int force, int *tile, int *blocks_per_cu, double *seconds);

/* ------------------------------------------------------ micro-benchmark -- */
/* Global memory -> LDS block copy on device `device` (the analogue of the
 * paper's DMA measurements, Sec. 6 / Eq. 4): one workgroup of 256 threads
 * copies `bytes` bytes (16..32768, multiple of 16) starting `offset` bytes
 * (0..252, multiple of 4) past a 256-byte boundary into LDS, `reps` times
 * (1..1024), each from a fresh source block 1 MiB apart; 512 MB written
 * elsewhere just before keep the sources out of the Infinity Cache.
 * src_host: 1 MiB host pattern copied into every source block (NULL: zeros).
 * Outputs (host arrays of reps entries): cycles[r] = shader-clock cycles of
 * copy r between two barriers; sums[r] = sum mod 2^32 of the 32-bit words
 * that LDS held after copy r (a check that the bytes arrived).
 * Synchronous; allocates reps MiB + 512 MB of device memory for the call. */
wd_status wd_micro_lds_copy(int device, int bytes, int offset, int reps,
                            const void *src_host, unsigned long long *cycles,
                            unsigned *sums);

/* Streaming probe on device `device`: a kernel reads nread (1..8) arrays of
 * `bytes` bytes each (16-byte lanes, one element per thread) and, with
 * write = 1, writes their sum to one more array; nontemporal = 1 uses
 * streaming loads and stores.  *seconds = mean time of one pass over reps
 * passes (HIP events, after 3 warm-up passes).  The measured ceilings feed
 * the timing model (Eqs. 1-2).  Synchronous; allocates (nread + 1) * bytes. */
wd_status wd_micro_stream(int device, int nread, int write, int nontemporal,
                          size_t bytes, int reps, double *seconds);

/* Resident-data probe on device `device`: a persistent grid (8 workgroups of
 * 256 threads per CU, dealt round-robin over the XCDs) reads a zero-filled
 * buffer of `bytes` bytes (1 MiB .. 4 GiB, whole MiB) `passes` times per
 * launch, each block the same addresses on every pass (16-byte lanes,
 * cached loads), after one warming launch.  The buffer therefore comes from
 * the XCDs' L2 while an eighth of it fits in 4 MB, from the 256 MB Infinity
 * Cache while it fits there, else from HBM.  *seconds = time of one pass
 * (HIP events over reps launches).  These read bandwidths are the beta of
 * the L2, Infinity-Cache and HBM tasks of the timing model (Eqs. 1-2).
 * Synchronous; allocates `bytes` of device memory for the call. */
wd_status wd_micro_resident(int device, size_t bytes, int passes, int reps,
                            double *seconds);

/* --------------------------------------------------------------- misc --- */

const char *wd_status_string(int status);
const char *wd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WD_H */
