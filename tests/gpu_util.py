"""Helpers for the GPU tests: move canonical numpy fields through the library's
pack/unpack and compare with the oracle.  Only marshalling, no arithmetic of
the method."""
import numpy as np
import torch

import paper_0710_2442_amd as wd

DEV = "cuda:0"


def to_field(g, psi, prec="f64", parity=wd.WD_FULL):
    """Canonical complex128 numpy spinor -> device field (full or one parity)."""
    canon = torch.from_numpy(np.ascontiguousarray(psi).reshape(-1)).to(DEV)
    f = wd.wd_new_field(g.dims, prec, 1, parity)
    wd.wd_spinor_pack(g, canon, f, parity, prec)
    return f


def from_field(g, f, prec="f64", parity=wd.WD_FULL):
    """Device field -> canonical complex128 numpy spinor (sites of other parity = 0)."""
    L1, L2, L3, L4 = g.dims
    canon = torch.zeros(L1 * L2 * L3 * L4 * 12, dtype=torch.complex128, device=DEV)
    wd.wd_spinor_unpack(g, f, canon, parity, prec)
    torch.cuda.synchronize()
    return canon.cpu().numpy().reshape(L4, L3, L2, L1, 4, 3)


def half_view(f, g, prec, which):
    """Tensor view of the even (0) or odd (1) half of a full field."""
    hb = wd.wd_field_bytes(g.dims, prec, 1, wd.WD_EVEN)
    return f[which * hb:(which + 1) * hb]


def rel_err(got, want):
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


# Per-site bars on the real components, relative to the site's largest
# |real| of the expected value.  FP64 and FP32: the arithmetic.  BF16
# storage: a stored real has relative rounding error <= 2^-8, and the change
# of spin basis on unpacking, (a +- b)/sqrt 2, keeps each error below 2^-8
# of the larger of the two results.  FP16 with a per-site scale m: absolute
# error <= 2^-12 m per stored real, m <= sqrt 2 times the largest chiral
# |real|, and the basis change adds two errors / sqrt 2: <= 2^-11.  Both
# reduced-precision bars add room for the FP32 arithmetic before storing.
SITE_BARS = {"f64": 1e-13, "f32": 1e-6, "f16": 2.0 ** -11 + 4e-6, "bf16": 2.0 ** -8 + 4e-6}


def site_err(got, want):
    """max over sites of max |got - want| / max |want| over the 24 reals of the
    site; sites where want is exactly zero must be exactly zero in got (else
    the result is inf)."""
    g = np.asarray(got).reshape(-1, 12)
    w = np.asarray(want).reshape(-1, 12)
    d = np.maximum(np.abs(g.real - w.real), np.abs(g.imag - w.imag)).max(axis=1)
    m = np.maximum(np.abs(w.real), np.abs(w.imag)).max(axis=1)
    nz = m > 0
    if np.any(d[~nz] != 0):
        return float("inf")
    return float((d[nz] / m[nz]).max()) if nz.any() else 0.0


def assert_close(got, want, prec=None, l2=None, site=None, what=""):
    """Whole-field relative L2 difference <= l2 AND per-site difference
    (site_err) <= site; the bars default to the precision's."""
    l2 = BARS_L2[prec] if l2 is None else l2
    site = SITE_BARS[prec] if site is None else site
    e2, es = rel_err(got, want), site_err(got, want)
    print(f"  parity {what}: rel L2 {e2:.3e} (bar {l2:.1e}), per-site {es:.3e} (bar {site:.1e})", flush=True)
    assert e2 <= l2, (what, e2, l2)
    assert es <= site, (what, es, site)


BARS_L2 = {"f64": 1e-13, "f32": 1e-6, "f16": 1e-3, "bf16": 2.0 ** -8}


def round_c64(a):
    return a.astype(np.complex64).astype(np.complex128)


R = 0.70710678118654752440


def to_storage_basis(psi):
    """The library stores spin in the basis where gamma_4 is diagonal:
    spins (0,1) <- (a + b) * r, spins (2,3) <- (a - b) * r, a = spins (0,1),
    b = spins (2,3), r = 1/sqrt 2 (the map is its own inverse)."""
    a = psi[..., 0:2, :]
    b = psi[..., 2:4, :]
    return np.concatenate([(a + b) * R, (a - b) * R], axis=-2)


def storage_round(psi, prec):
    """psi as the GPU sees it after storing it in `prec` (rounding happens in
    the storage basis), returned in the chiral basis."""
    from oracle import solvers
    t = to_storage_basis(psi)
    if prec == "f64":
        r = t
    elif prec == "f32":
        r = t.astype(np.complex64).astype(np.complex128)
    else:
        r = solvers.round_storage(t, prec).astype(np.complex128)
    return to_storage_basis(r)
