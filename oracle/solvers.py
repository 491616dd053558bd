"""Krylov solvers for D_W x = b, written out plainly (test infrastructure only).

The paper leaves the solver that applies Eq. 3 over and over unspecified
(Sec. 5, data in on-chip memory).  The readings used throughout:

* CGLS: CG on the normal equations D^dag D x = D^dag b, started from x = 0,
  with the recursive residual s = b - D x carried explicitly so that the
  stopping test is on |s| / |b|.
* even-odd CGLS: CGLS on the Schur operator M = 1 - k^2 H_eo H_oe of the even
  sites, right-hand side b_e + k H_eo b_o, then x_o = b_o + k H_oe x_e.  With
  that x_o the full residual vanishes on odd sites and equals M's residual on
  even sites.
* defect correction: FP64 outer loop r = b - D x, inner solve of D e = r/|r|
  in reduced precision to a loose tolerance, x += |r| e, repeat.
* FGCR(m): flexible GCR with a right preconditioner, modified Gram-Schmidt,
  restart after m directions with the FP64 true residual; falls back to CGLS
  when the residual stagnates or stops being finite.

Convergence of every solver is judged on the true residual |b - D x|/|b|.
"""
from __future__ import annotations

import numpy as np

from . import wilson


def vdot(a, b):
    """<a, b> = sum conj(a) b (complex, FP64)."""
    return np.vdot(a.ravel(), b.ravel())


def norm2(a):
    return float(np.vdot(a.ravel(), a.ravel()).real)


def cgls(A, Adag, b, tol, maxiter=100000, x0=None):
    """CG on the normal equations of A x = b.

    Returns (x, iterations, [|s_k|/|b| history]).  Stops when the recursive
    residual |s| <= tol |b|.
    """
    bn = np.sqrt(norm2(b))
    if bn == 0.0:
        return np.zeros_like(b), 0, [0.0]
    x = np.zeros_like(b) if x0 is None else x0.copy()
    s = b - A(x) if x0 is not None else b.copy()
    r = Adag(s)
    p = r.copy()
    gamma = norm2(r)
    hist = [np.sqrt(norm2(s)) / bn]
    k = 0
    while hist[-1] > tol and k < maxiter:
        q = A(p)
        alpha = gamma / norm2(q)
        x = x + alpha * p
        s = s - alpha * q
        r = Adag(s)
        gamma_new = norm2(r)
        beta = gamma_new / gamma
        gamma = gamma_new
        p = r + beta * p
        k += 1
        hist.append(np.sqrt(norm2(s)) / bn)
    return x, k, hist


def true_residual(U, b, x, kappa, tbc=-1):
    """|b - D_W x| / |b| in FP64."""
    bn = np.sqrt(norm2(b))
    if bn == 0.0:
        return 0.0
    return np.sqrt(norm2(b - wilson.dirac(U, x, kappa, tbc))) / bn


def solve_cgls_full(U, b, kappa, tol, tbc=-1, maxiter=100000):
    """CGLS on the full lattice operator D_W."""
    A = lambda v: wilson.dirac(U, v, kappa, tbc)
    Ad = lambda v: wilson.dirac(U, v, kappa, tbc, dagger=True)
    return cgls(A, Ad, b, tol, maxiter)


def eo_rhs(U, b, kappa, p=0, tbc=-1):
    """b_p + k H_{p,1-p} b_{1-p} (supported on parity p)."""
    dims = wilson.dims_of(b)
    mp = wilson.parity_mask(dims, p)
    return mp * b + kappa * wilson.hop_parity(U, b, p, tbc)


def eo_reconstruct(U, b, x_p, kappa, p=0, tbc=-1):
    """Full solution from the parity-p part: x_q = b_q + k H_{q,p} x_p."""
    dims = wilson.dims_of(b)
    q = 1 - p
    mq = wilson.parity_mask(dims, q)
    return wilson.parity_mask(dims, p) * x_p + mq * b + kappa * wilson.hop_parity(U, x_p, q, tbc)


def solve_eo_cgls(U, b, kappa, tol, p=0, tbc=-1, maxiter=100000):
    """Even-odd preconditioned CGLS.  Returns (x_full, iterations, history).

    The history is the Schur residual relative to |b| (full field), which in
    exact arithmetic equals the full-lattice relative residual.
    """
    bn = np.sqrt(norm2(b))
    if bn == 0.0:
        return np.zeros_like(b), 0, [0.0]
    bh = eo_rhs(U, b, kappa, p, tbc)
    A = lambda v: wilson.schur(U, v, kappa, p, tbc)
    Ad = lambda v: wilson.schur(U, v, kappa, p, tbc, dagger=True)
    # stop on |s| / |b| rather than |s| / |bh|
    x_p, k, hist = cgls(A, Ad, bh, tol * bn / np.sqrt(norm2(bh)), maxiter)
    scale = np.sqrt(norm2(bh)) / bn
    hist = [h * scale for h in hist]
    return eo_reconstruct(U, b, x_p, kappa, p, tbc), k, hist


# ----------------------------------------------------------------------------
# reduced-precision storage emulation (used by the defect-correction oracle)


def round_bf16(a):
    """Round float32 values to bfloat16 (nearest, ties to even), back as float32."""
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def round_storage(psi, storage):
    """Round a complex field as it would be stored in ``storage`` precision.

    'f32' rounds to complex64; 'bf16' rounds each real to bfloat16; 'f16'
    divides each site by its largest |real| (kept in float32), rounds to
    IEEE half and multiplies back.
    """
    c = psi.astype(np.complex64)
    if storage == "f32":
        return c
    re = c.real.astype(np.float32)
    im = c.imag.astype(np.float32)
    if storage == "bf16":
        return (round_bf16(re) + 1j * round_bf16(im)).astype(np.complex64)
    if storage == "f16":
        site_axes = (-2, -1)
        m = np.maximum(np.abs(re).max(axis=site_axes), np.abs(im).max(axis=site_axes))
        m = m.astype(np.float32)
        inv = np.where(m > 0, np.float32(1.0) / np.where(m > 0, m, 1), 0).astype(np.float32)
        re16 = (re * inv[..., None, None]).astype(np.float16).astype(np.float32)
        im16 = (im * inv[..., None, None]).astype(np.float16).astype(np.float32)
        return ((re16 * m[..., None, None]) + 1j * (im16 * m[..., None, None])).astype(np.complex64)
    raise ValueError(storage)


def _cgls_lowprec(A, Adag, b, tol, maxiter, storage):
    """CGLS in float32 arithmetic with vectors rounded to ``storage`` between steps.

    Inner products and norms are accumulated in FP64.
    """
    b = round_storage(b, storage)
    bn = np.sqrt(norm2(b.astype(np.complex128)))
    x = np.zeros_like(b, dtype=np.complex64)
    s = b.copy()
    r = round_storage(Adag(s), storage)
    p = r.copy()
    gamma = norm2(r.astype(np.complex128))
    k = 0
    while k < maxiter:
        q = round_storage(A(p), storage)
        qq = norm2(q.astype(np.complex128))
        if not np.isfinite(qq) or qq <= 0:
            break
        alpha = np.float32(gamma / qq)
        x = (x + alpha * p).astype(np.complex64)
        s = round_storage(s - alpha * q, storage)
        k += 1
        if np.sqrt(norm2(s.astype(np.complex128))) <= tol * bn:
            break
        r = round_storage(Adag(s), storage)
        gamma_new = norm2(r.astype(np.complex128))
        beta = np.float32(gamma_new / gamma)
        gamma = gamma_new
        p = round_storage(r + beta * p, storage)
    return x, k


def solve_defect_correction(U, b, kappa, tol, inner_tol=1e-3, storage="f32",
                            tbc=-1, max_outer=100, inner_maxiter=10000):
    """FP64 defect correction around an emulated reduced-precision eo-CGLS.

    Outer (FP64): r = b - D x; stop when |r|/|b| <= tol; otherwise solve
    D e = r/|r| with the inner solver in float32 arithmetic (links rounded to
    complex64, vectors rounded to ``storage``), and accumulate x += |r| e in
    FP64.  Returns (x, outer iterations, total inner iterations).
    """
    U32 = U.astype(np.complex64)
    bn = np.sqrt(norm2(b))
    x = np.zeros_like(b)
    total_inner = 0
    for outer in range(max_outer + 1):
        r = b - wilson.dirac(U, x, kappa, tbc)
        rn = np.sqrt(norm2(r))
        if rn <= tol * bn:
            return x, outer, total_inner
        if outer == max_outer:
            break
        rh = (r / rn).astype(np.complex64)
        k32 = np.float32(kappa)
        bh = eo_rhs(U32, rh, k32, 0, tbc).astype(np.complex64)
        A = lambda v: wilson.schur(U32, v, k32, 0, tbc).astype(np.complex64)
        Ad = lambda v: wilson.schur(U32, v, k32, 0, tbc, dagger=True).astype(np.complex64)
        xe, k = _cgls_lowprec(A, Ad, bh, inner_tol, inner_maxiter, storage)
        total_inner += k
        e = eo_reconstruct(U32, rh, xe, k32, 0, tbc)
        x = x + rn * e.astype(np.complex128)
    return x, max_outer, total_inner


# ----------------------------------------------------------------------------
# flexible GCR with a right preconditioner


def fgcr(Dop, precond, b, tol, m=16, maxiter=2000, stagnation=25, cg_fallback=None):
    """FGCR(m): z_k = N(r), w_k = D z_k, MGS against earlier w_j (same ops on z_j),
    x += a z_k, r -= a w_k with a = <w_k, r>/<w_k, w_k>.

    After m directions the basis is dropped and r is recomputed as b - D x.
    If |r| has not fallen below 0.99x its best value within ``stagnation``
    iterations, or becomes non-finite, ``cg_fallback(x, r)`` (returning the
    correction e with D e ~= r) finishes the solve.
    Returns (x, iterations, fallback_used, history).
    """
    bn = np.sqrt(norm2(b))
    x = np.zeros_like(b)
    r = b.copy()
    hist = [1.0]
    it = 0
    best = np.inf
    since_best = 0
    while it < maxiter:
        W, Z = [], []
        for _ in range(m):
            z = precond(r)
            w = Dop(z)
            for wj, zj in zip(W, Z):
                c = vdot(wj, w)
                w = w - c * wj
                z = z - c * zj
            nw = np.sqrt(norm2(w))
            bad = (not np.isfinite(nw)) or nw == 0.0
            if not bad:
                w = w / nw
                z = z / nw
                a = vdot(w, r)
                x = x + a * z
                r = r - a * w
                W.append(w)
                Z.append(z)
            it += 1
            rel = np.sqrt(norm2(r)) / bn
            hist.append(rel)
            if rel < 0.99 * best:
                best = rel
                since_best = 0
            else:
                since_best += 1
            if bad or not np.isfinite(rel) or since_best >= stagnation:
                if cg_fallback is None:
                    return x, it, False, hist
                r = b - Dop(x)
                x = x + cg_fallback(x, r)
                return x, it, True, hist
            if rel <= tol:
                r_true = b - Dop(x)
                if np.sqrt(norm2(r_true)) / bn <= tol:
                    return x, it, False, hist
                r = r_true
                break
        # restart with the true residual
        r = b - Dop(x)
    return x, it, False, hist
