"""The Wilson-Dirac hopping term of Eq. 3 and the operators built on it.

Test infrastructure only (see the package docstring).

Conventions (the paper gives Eq. 3 and nothing else about the operator):

* hopping term, Eq. 3 (Sec. 5):
      (H psi)_x = sum_mu { U_{x,mu} (1 + gamma_mu) psi_{x+mu}
                           + U^dag_{x-mu,mu} (1 - gamma_mu) psi_{x-mu} }
  with (1 + gamma_mu) on the forward hop, literally as printed.
* Wilson-Dirac operator in hopping form: D_W = 1 - kappa * H.
* boundary: periodic in x1..x3; the time direction x4 carries a factor
  ``tbc`` (-1 = antiperiodic) on every hop that crosses x4 = L4-1 <-> 0.
* even-odd: parity(x) = (x1+x2+x3+x4) mod 2.  The parity-restricted hop
  H_{p,1-p} is mask_p . H . mask_{1-p}, computed by masking the full
  operator (no checkerboard index is used here).

Fields are arrays in the canonical layout of ``synthetic``:
spinor (L4,L3,L2,L1,4,3), gauge (L4,L3,L2,L1,4,3,3).  mu = 0..3 stands for
the directions x1..x4.
"""
from __future__ import annotations

import numpy as np

from .gamma import GAMMA, GAMMA5, ID4

# numpy axis of the (L4, L3, L2, L1, ...) array that direction mu runs along
MU_AXIS = (3, 2, 1, 0)


def dims_of(field):
    L4, L3, L2, L1 = field.shape[:4]
    return (L1, L2, L3, L4)


def shift_forward(f, mu, tbc=-1):
    """g_x = f_{x+mu}, with the time-boundary factor on the wrapped slice."""
    g = np.roll(f, -1, axis=MU_AXIS[mu])
    if mu == 3 and tbc != 1:
        g[-1] = g[-1] * tbc
    return g


def shift_backward(f, mu, tbc=-1):
    """g_x = f_{x-mu}, with the time-boundary factor on the wrapped slice."""
    g = np.roll(f, 1, axis=MU_AXIS[mu])
    if mu == 3 and tbc != 1:
        g[0] = g[0] * tbc
    return g


def spin_mul(S, psi):
    """Apply a 4x4 spin matrix to every site: (S psi)_{s,a} = sum_t S_st psi_{t,a}."""
    return np.einsum("st,...ta->...sa", S, psi)


def colour_mul(U, psi):
    """(U psi)_{s,a} = sum_b U_ab psi_{s,b} at every site."""
    return np.einsum("...ab,...sb->...sa", U, psi)


def colour_mul_dag(U, psi):
    """(U^dag psi)_{s,a} = sum_b conj(U_ba) psi_{s,b} at every site."""
    return np.einsum("...ba,...sb->...sa", np.conj(U), psi)


def hop(U, psi, tbc=-1, dagger=False):
    """Eq. 3: H psi over the whole lattice.

    ``dagger=True`` applies the adjoint H^dag.  Because gamma_mu is Hermitian,
    the adjoint of the forward term U_{x,mu}(1+gamma_mu) psi_{x+mu} is the
    backward term with (1+gamma_mu); so H^dag is Eq. 3 with the two
    projectors exchanged.
    """
    s = -1.0 if dagger else 1.0
    out = np.zeros_like(psi)
    for mu in range(4):
        Umu = U[..., mu, :, :]
        fwd = shift_forward(psi, mu, tbc)
        out += colour_mul(Umu, spin_mul(ID4 + s * GAMMA[mu], fwd))
        U_back = shift_backward(Umu, mu, 1)  # U_{x-mu,mu}
        bwd = shift_backward(psi, mu, tbc)
        out += colour_mul_dag(U_back, spin_mul(ID4 - s * GAMMA[mu], bwd))
    return out


def dirac(U, psi, kappa, tbc=-1, dagger=False):
    """D_W psi = psi - kappa * H psi (or D_W^dag with ``dagger``)."""
    return psi - kappa * hop(U, psi, tbc, dagger)


def gamma5(psi):
    return spin_mul(GAMMA5, psi)


def parity_field(dims):
    """(x1+x2+x3+x4) mod 2 on the (L4,L3,L2,L1) grid."""
    L1, L2, L3, L4 = dims
    x4, x3, x2, x1 = np.meshgrid(
        np.arange(L4), np.arange(L3), np.arange(L2), np.arange(L1), indexing="ij"
    )
    return (x1 + x2 + x3 + x4) % 2


def parity_mask(dims, p):
    """1.0 on sites of parity p, 0.0 elsewhere, broadcastable to a spinor."""
    return (parity_field(dims) == p).astype(np.float64)[..., None, None]


def hop_parity(U, psi, p, tbc=-1, dagger=False):
    """H_{p,1-p} psi = mask_p H (mask_{1-p} psi): output on parity p only."""
    dims = dims_of(psi)
    return parity_mask(dims, p) * hop(U, parity_mask(dims, 1 - p) * psi, tbc, dagger)


def schur(U, psi, kappa, p=0, tbc=-1, dagger=False):
    """Even-odd Schur complement on parity p:  M = 1 - kappa^2 H_{p,1-p} H_{1-p,p}.

    With D_W = [[1, -k H_pq], [-k H_qp, 1]] (q = 1-p), eliminating the q sites
    gives (1 - k^2 H_pq H_qp) x_p = b_p + k H_pq b_q and x_q = b_q + k H_qp x_p.
    ``dagger`` gives M^dag = 1 - k^2 H_qp^dag H_pq^dag (restricted to parity p),
    i.e. the same product with both hops adjointed.
    """
    dims = dims_of(psi)
    psi = parity_mask(dims, p) * psi
    t = hop_parity(U, psi, 1 - p, tbc, dagger)
    return psi - kappa * kappa * hop_parity(U, t, p, tbc, dagger)


def hop_sites(U, psi, sites, tbc=-1):
    """Eq. 3 evaluated one site at a time, for sampled checks on big lattices.

    ``sites`` is a sequence of (x1, x2, x3, x4).  Returns (n, 4, 3).
    """
    L1, L2, L3, L4 = dims_of(psi)
    L = (L1, L2, L3, L4)
    out = np.zeros((len(sites), 4, 3), dtype=np.complex128)
    for n, x in enumerate(sites):
        x = list(x)
        acc = np.zeros((4, 3), dtype=np.complex128)
        for mu in range(4):
            xf = list(x)
            xf[mu] = (x[mu] + 1) % L[mu]
            sf = tbc if (mu == 3 and x[3] == L4 - 1) else 1.0
            xb = list(x)
            xb[mu] = (x[mu] - 1) % L[mu]
            sb = tbc if (mu == 3 and x[3] == 0) else 1.0
            Uf = U[x[3], x[2], x[1], x[0], mu]
            Ub = U[xb[3], xb[2], xb[1], xb[0], mu]
            pf = psi[xf[3], xf[2], xf[1], xf[0]]
            pb = psi[xb[3], xb[2], xb[1], xb[0]]
            acc += sf * (Uf @ ((ID4 + GAMMA[mu]) @ pf).T).T
            acc += sb * (np.conj(Ub).T @ ((ID4 - GAMMA[mu]) @ pb).T).T
        out[n] = acc
    return out


def dense_hop(U, tbc=-1):
    """Brute-force (12V x 12V) matrix of Eq. 3, assembled site by site.

    Row/column index = 12*idx + 3*spin + colour with the canonical site index
    idx = x1 + L1*(x2 + L2*(x3 + L3*x4)).  On a lattice with an extent of 2
    the forward and backward neighbours coincide and their blocks add.
    """
    L1, L2, L3, L4 = dims_of(U)
    L = (L1, L2, L3, L4)
    V = L1 * L2 * L3 * L4

    def index(x):
        return x[0] + L1 * (x[1] + L2 * (x[2] + L3 * x[3]))

    H = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    for x4 in range(L4):
        for x3 in range(L3):
            for x2 in range(L2):
                for x1 in range(L1):
                    x = (x1, x2, x3, x4)
                    i = index(x)
                    for mu in range(4):
                        xf = list(x)
                        xf[mu] = (x[mu] + 1) % L[mu]
                        sf = tbc if (mu == 3 and x4 == L4 - 1) else 1.0
                        j = index(xf)
                        Uf = U[x4, x3, x2, x1, mu]
                        H[12 * i:12 * i + 12, 12 * j:12 * j + 12] += sf * np.kron(
                            ID4 + GAMMA[mu], Uf
                        )
                        xb = list(x)
                        xb[mu] = (x[mu] - 1) % L[mu]
                        sb = tbc if (mu == 3 and x4 == 0) else 1.0
                        j = index(xb)
                        Ub = U[xb[3], xb[2], xb[1], xb[0], mu]
                        H[12 * i:12 * i + 12, 12 * j:12 * j + 12] += sb * np.kron(
                            ID4 - GAMMA[mu], np.conj(Ub).T
                        )
    return H


def dense_dirac(U, kappa, tbc=-1):
    H = dense_hop(U, tbc)
    return np.eye(H.shape[0], dtype=np.complex128) - kappa * H


def flat(psi):
    """Canonical spinor -> vector ordered like the dense matrix's columns."""
    return psi.reshape(-1)


def unflat(v, dims):
    L1, L2, L3, L4 = dims
    return v.reshape(L4, L3, L2, L1, 4, 3)


def gauge_transform(U, psi, Omega, tbc=-1):
    """U'_{x,mu} = Omega_x U_{x,mu} Omega^dag_{x+mu},  psi'_x = Omega_x psi_x.

    ``Omega`` has shape (L4,L3,L2,L1,3,3).  The time-boundary factor belongs
    to the hop, not to the links, so it plays no part here.
    """
    Up = np.empty_like(U)
    for mu in range(4):
        Om_f = np.roll(Omega, -1, axis=MU_AXIS[mu])
        Up[..., mu, :, :] = Omega @ U[..., mu, :, :] @ np.conj(np.swapaxes(Om_f, -1, -2))
    psip = colour_mul(Omega, psi)
    return Up, psip
