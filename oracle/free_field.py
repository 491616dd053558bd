"""Unit-link (free-field) closed forms for D_W = 1 - kappa*H with Eq. 3's H.

Test infrastructure only.

With U = 1 and psi_x = exp(i p.x) u, where p_mu = 2 pi n_mu / L_mu in space
and p_4 = 2 pi (n_4 + 1/2) / L_4 in the antiperiodic time direction,
Eq. 3 gives  H psi = sum_mu [(1+g_mu) e^{i p_mu} + (1-g_mu) e^{-i p_mu}] psi,
so
    D_W psi = [A(p) - 2 i kappa sum_mu g_mu sin p_mu] psi,
    A(p)    = 1 - 2 kappa sum_mu cos p_mu.
Because (sum g_mu s_mu)^2 = sum s_mu^2, the inverse of that 4x4 symbol is
    [A + 2 i kappa sum g_mu s_mu] / (A^2 + 4 kappa^2 sum s_mu^2),
and the eigenvalues are A +- 2 i kappa sqrt(sum s_mu^2), each six-fold
(two spin directions x three colours).
"""
from __future__ import annotations

import numpy as np

from .gamma import GAMMA, ID4


def momenta(dims, tbc=-1):
    """Allowed momenta per direction: 2 pi n / L (+ pi/L in time if antiperiodic)."""
    ps = []
    for mu, L in enumerate(dims):
        n = np.arange(L)
        shift = 0.5 if (mu == 3 and tbc == -1) else 0.0
        ps.append(2.0 * np.pi * (n + shift) / L)
    return ps


def plane_wave(dims, p, u):
    """psi_x = exp(i p.x) u, u of shape (4,3); canonical layout."""
    L1, L2, L3, L4 = dims
    x4, x3, x2, x1 = np.meshgrid(
        np.arange(L4), np.arange(L3), np.arange(L2), np.arange(L1), indexing="ij"
    )
    phase = np.exp(1j * (p[0] * x1 + p[1] * x2 + p[2] * x3 + p[3] * x4))
    return phase[..., None, None] * np.asarray(u)[None, None, None, None]


def momentum_of(dims, n, tbc=-1):
    """p_mu = 2 pi n_mu / L_mu, plus pi / L_4 in an antiperiodic time direction."""
    return [2.0 * np.pi * (n[mu] + (0.5 if (mu == 3 and tbc == -1) else 0.0)) / dims[mu] for mu in range(4)]


def plane_wave_n(dims, n, u, tbc=-1):
    """The plane wave of integer momentum numbers n (momentum_of(dims, n, tbc))
    with its phase reduced exactly: p.x / 2 pi = sum_mu k_mu x_mu / (2 L_mu),
    k_mu = 2 n_mu (+ 1 in antiperiodic time), is a fraction with denominator
    D = 2 lcm(L); its numerator is taken mod D in integers, so the rounding of
    the phase stays ~1e-16 however large p.x is (unreduced, p.x reaches
    hundreds on a 32^3x64 lattice and its rounding alone is ~3e-14)."""
    L1, L2, L3, L4 = dims
    D = 2 * int(np.lcm.reduce([int(L) for L in dims]))
    k = [2 * int(n[mu]) + (1 if (mu == 3 and tbc == -1) else 0) for mu in range(4)]
    w = [k[mu] * (D // (2 * int(dims[mu]))) for mu in range(4)]
    x4, x3, x2, x1 = np.meshgrid(
        np.arange(L4), np.arange(L3), np.arange(L2), np.arange(L1), indexing="ij"
    )
    num = (w[0] * x1 + w[1] * x2 + w[2] * x3 + w[3] * x4) % D
    phase = np.exp(2j * np.pi * (num / D))
    return phase[..., None, None] * np.asarray(u)[None, None, None, None]


def symbol(p, kappa):
    """4x4 spin matrix that D_W multiplies a plane wave of momentum p by."""
    A = 1.0 - 2.0 * kappa * sum(np.cos(pm) for pm in p)
    S = sum(GAMMA[mu] * np.sin(p[mu]) for mu in range(4))
    return A * ID4 - 2j * kappa * S


def spectrum(dims, kappa, tbc=-1):
    """All 12V free-field eigenvalues of D_W (each pair value is 6-fold)."""
    ps = momenta(dims, tbc)
    P = np.meshgrid(*ps, indexing="ij")
    A = 1.0 - 2.0 * kappa * sum(np.cos(q) for q in P)
    s = np.sqrt(sum(np.sin(q) ** 2 for q in P))
    lam_p = (A + 2j * kappa * s).ravel()
    lam_m = (A - 2j * kappa * s).ravel()
    return np.concatenate([np.repeat(lam_p, 6), np.repeat(lam_m, 6)])


def solve(b, kappa, tbc=-1):
    """Exact D_W^{-1} b for unit links, through the lattice Fourier transform.

    phi_x = exp(-i pi x4 / L4) b_x is periodic when tbc = -1, so an ordinary
    FFT diagonalises the operator; every momentum is inverted with the
    closed-form inverse of the 4x4 symbol above.
    """
    L4, L3, L2, L1 = b.shape[:4]
    dims = (L1, L2, L3, L4)
    x4 = np.arange(L4).reshape(L4, 1, 1, 1, 1, 1)
    shift = 0.5 if tbc == -1 else 0.0
    tw = np.exp(-1j * 2.0 * np.pi * shift * x4 / L4)
    bt = np.fft.fftn(b * tw, axes=(0, 1, 2, 3))
    # momentum grids on the (L4,L3,L2,L1) axes
    p1 = 2 * np.pi * np.fft.fftfreq(L1) * 1.0
    p2 = 2 * np.pi * np.fft.fftfreq(L2)
    p3 = 2 * np.pi * np.fft.fftfreq(L3)
    p4 = 2 * np.pi * (np.fft.fftfreq(L4) + shift / L4)
    P4, P3, P2, P1 = np.meshgrid(p4, p3, p2, p1, indexing="ij")
    P = (P1, P2, P3, P4)
    A = 1.0 - 2.0 * kappa * sum(np.cos(q) for q in P)
    S = [np.sin(q) for q in P]
    den = A * A + 4.0 * kappa * kappa * sum(s * s for s in S)
    # numerator matrix (A + 2 i k sum g s) applied on spin
    num = np.einsum("...,st->...st", A, ID4) + 2j * kappa * sum(
        np.einsum("...,st->...st", S[mu], GAMMA[mu]) for mu in range(4)
    )
    xt = np.einsum("...st,...tc->...sc", num, bt) / den[..., None, None]
    x = np.fft.ifftn(xt, axes=(0, 1, 2, 3)) / tw
    return x


def lambda_min_normal(dims, kappa, tbc=-1):
    """Smallest eigenvalue of D^dag D for unit links: min_p A^2 + 4k^2 sum s^2."""
    ps = momenta(dims, tbc)
    P = np.meshgrid(*ps, indexing="ij")
    A = 1.0 - 2.0 * kappa * sum(np.cos(q) for q in P)
    s2 = sum(np.sin(q) ** 2 for q in P)
    vals = A * A + 4 * kappa * kappa * s2
    return float(vals.min()), float(vals.max())
