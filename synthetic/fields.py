"""Seeded generators for gauge links, spinor sources and gauge transformations.

Recipe (all draws from ``numpy.random.Generator(PCG64(seed))``):

* gauge link U_{x,mu} = exp(i*eps*H) with H a random traceless Hermitian 3x3
  matrix: A_ij = N(0,1) + i N(0,1),  H = (A + A^dag)/2 - tr(.)/3.  The
  exponential is taken through the eigen-decomposition of H.  The result is
  re-unitarised (Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1)), so
  every link is in SU(3) to rounding and its third row is exactly the one a
  two-row compression rebuilds.  Links are drawn in site order, then mu.
* Gaussian spinor: real and imaginary parts of the 12 spin-colour components
  are independent N(0,1).
* point source: delta_{x,0} delta_{s,s0} delta_{c,c0}.
* random SU(3) gauge transformation: Haar-distributed via QR of a complex
  Gaussian matrix with the phase of R's diagonal removed, then det fixed to 1.
"""
from __future__ import annotations

import numpy as np

# Seeds of the named workloads: gauge = 1000 + n (+ lattice index for the
# eight-lattice batch), source = 2000 + n.
CONFIG_SEEDS = {
    "wilson_8x8x8x8": (1001, 2001),
    "dslash_32x32x32x64": (1002, 2002),
    "mixed_32x32x32x64": (1003, 2003),
    "mrhs_24x24x24x48": (1004, 2004),
    "ptc_16x16x16x16": (1005, 2005),
}

# Eight lattices of uneven size solved in one batched launch, with the link
# roughness assigned cyclically from {0.2, 0.3, 0.4} in the listed order.
_BATCH_DIMS = [
    (8, 8, 8, 8),
    (12, 12, 12, 12),
    (16, 16, 16, 32),
    (16, 16, 16, 16),
    (20, 20, 20, 40),
    (12, 12, 12, 24),
    (16, 16, 16, 24),
    (8, 8, 8, 16),
]
_BATCH_EPS = (0.2, 0.3, 0.4)


def batch_lattices():
    """[(dims, eps, gauge_seed)] of the eight-lattice batch (689,408 sites)."""
    return [(d, _BATCH_EPS[i % 3], 1004 + i) for i, d in enumerate(_BATCH_DIMS)]


def lattice_shape(dims):
    """numpy shape (L4, L3, L2, L1) for dims = (L1, L2, L3, L4)."""
    L1, L2, L3, L4 = (int(d) for d in dims)
    return (L4, L3, L2, L1)


def volume(dims):
    return int(np.prod([int(d) for d in dims]))


def rng_for(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def random_traceless_hermitian(rng, n):
    """n random traceless Hermitian 3x3 matrices with Gaussian entries."""
    z = rng.standard_normal((n, 3, 3, 2))
    A = z[..., 0] + 1j * z[..., 1]
    H = 0.5 * (A + np.conj(np.swapaxes(A, -1, -2)))
    tr = np.trace(H, axis1=-2, axis2=-1).real / 3.0
    H = H - tr[:, None, None] * np.eye(3)
    return H


def _reunitarise(M):
    """Gram-Schmidt rows 0,1; row 2 = conj(row0 x row1).  In place, returns M."""
    r0 = M[:, 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = M[:, 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    M[:, 0, :] = r0
    M[:, 1, :] = r1
    M[:, 2, :] = r2
    return M


def _expi(H, eps):
    w, V = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    return np.einsum("nab,nb,ncb->nac", V, ph, np.conj(V))


def gauge_field(dims, eps, seed, chunk=1 << 18):
    """Random near-unit SU(3) links, shape (L4,L3,L2,L1,4,3,3) complex128."""
    V = volume(dims)
    rng = rng_for(seed)
    out = np.empty((V * 4, 3, 3), dtype=np.complex128)
    n = V * 4
    for a in range(0, n, chunk):
        m = min(chunk, n - a)
        H = random_traceless_hermitian(rng, m)
        out[a:a + m] = _reunitarise(_expi(H, eps))
    return out.reshape(lattice_shape(dims) + (4, 3, 3))


def unit_gauge(dims):
    shp = lattice_shape(dims) + (4, 3, 3)
    U = np.zeros(shp, dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def random_su3(n, seed):
    """n Haar-random SU(3) matrices (for gauge-covariance checks)."""
    rng = rng_for(seed)
    z = rng.standard_normal((n, 3, 3, 2))
    A = (z[..., 0] + 1j * z[..., 1]) / np.sqrt(2.0)
    Q, R = np.linalg.qr(A)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    Q = Q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(Q)
    Q = Q / (det ** (1.0 / 3.0))[:, None, None]
    return Q


def gaussian_spinor(dims, seed, nrhs=None):
    """Gaussian spinor field (L4,L3,L2,L1,4,3) complex128 (leading nrhs axis if given)."""
    rng = rng_for(seed)
    shp = lattice_shape(dims) + (4, 3)
    if nrhs is not None:
        shp = (int(nrhs),) + shp
    z = rng.standard_normal(shp + (2,))
    return z[..., 0] + 1j * z[..., 1]


def point_source(dims, spin, colour, site=(0, 0, 0, 0)):
    psi = np.zeros(lattice_shape(dims) + (4, 3), dtype=np.complex128)
    x1, x2, x3, x4 = site
    psi[x4, x3, x2, x1, spin, colour] = 1.0
    return psi


def point_sources(dims, site=(0, 0, 0, 0)):
    """The 12 spin-colour point sources at one site, shape (12, L4,L3,L2,L1,4,3)."""
    return np.stack([point_source(dims, s, c, site) for s in range(4) for c in range(3)])
