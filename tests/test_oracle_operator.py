"""Pins of the oracle's Wilson-Dirac operator against facts it does not encode.

Each test checks the oracle against something the paper or the mathematics
fixes independently of how the oracle is written: the Clifford algebra, the
closed-form action of the free operator on plane waves (which fixes the sign
of the projectors and the time boundary), the free spectrum, a brute-force
dense matrix assembled site by site, gamma5-hermiticity, gauge covariance
and the trivial kappa = 0 case.
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import free_field, wilson
from oracle.gamma import GAMMA, GAMMA5, ID4


def test_gamma_algebra():
    for mu in range(4):
        assert np.allclose(GAMMA[mu], GAMMA[mu].conj().T)
        for nu in range(4):
            ac = GAMMA[mu] @ GAMMA[nu] + GAMMA[nu] @ GAMMA[mu]
            assert np.allclose(ac, 2.0 * (mu == nu) * ID4)
    g5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
    assert np.allclose(g5, GAMMA5)
    assert np.allclose(GAMMA5, np.diag([1, 1, -1, -1]))


@pytest.mark.parametrize("dims", [(4, 4, 4, 6), (2, 4, 2, 6), (6, 4, 2, 4)])
@pytest.mark.parametrize("tbc", [-1, 1])
def test_plane_wave_closed_form(dims, tbc):
    """U = 1: D psi = [1 - 2k sum cos p - 2ik sum g sin p] psi for psi = e^{ipx} u."""
    rng = np.random.default_rng(7)
    kappa = 0.137
    U = syn.unit_gauge(dims)
    for _ in range(4):
        n = [rng.integers(0, L) for L in dims]
        p = [2 * np.pi * n[mu] / dims[mu] for mu in range(3)]
        p.append(2 * np.pi * (n[3] + (0.5 if tbc == -1 else 0.0)) / dims[3])
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi = free_field.plane_wave(dims, p, u)
        got = wilson.dirac(U, psi, kappa, tbc)
        S = free_field.symbol(p, kappa)
        want = free_field.plane_wave(dims, p, S @ u)
        assert np.max(np.abs(got - want)) < 1e-12


def test_plane_wave_rejects_wrong_boundary():
    """A periodic-time plane wave is not an eigenvector of the antiperiodic operator."""
    dims = (4, 4, 4, 6)
    U = syn.unit_gauge(dims)
    p = [0.0, 0.0, 0.0, 2 * np.pi / 6]
    u = np.ones((4, 3), dtype=complex)
    psi = free_field.plane_wave(dims, p, u)
    got = wilson.dirac(U, psi, 0.1, -1)
    want = free_field.plane_wave(dims, p, free_field.symbol(p, 0.1) @ u)
    assert np.max(np.abs(got - want)) > 1e-3


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 4, 2, 6)])
def test_free_spectrum_matches_dense(dims):
    kappa = 0.124
    D = wilson.dense_dirac(syn.unit_gauge(dims), kappa)
    ev = np.linalg.eigvals(D)
    want = free_field.spectrum(dims, kappa)
    key = lambda z: (np.round(z.real, 9), np.round(z.imag, 9))
    a = np.array(sorted(ev, key=key))
    b = np.array(sorted(want, key=key))
    assert np.max(np.abs(a - b)) < 1e-10


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 4, 2, 6), (4, 4, 4, 4)])
def test_dense_matches_matrix_free(dims):
    U = syn.gauge_field(dims, 0.5, 11)
    psi = syn.gaussian_spinor(dims, 12)
    H = wilson.dense_hop(U)
    got = wilson.flat(wilson.hop(U, psi))
    want = H @ wilson.flat(psi)
    assert np.max(np.abs(got - want)) < 1e-12


def test_sitewise_matches_matrix_free():
    dims = (4, 6, 4, 8)
    U = syn.gauge_field(dims, 0.4, 3)
    psi = syn.gaussian_spinor(dims, 4)
    full = wilson.hop(U, psi)
    sites = [(0, 0, 0, 0), (3, 5, 3, 7), (1, 2, 3, 0), (2, 0, 1, 7), (3, 3, 0, 4)]
    got = wilson.hop_sites(U, psi, sites)
    for n, (x1, x2, x3, x4) in enumerate(sites):
        assert np.max(np.abs(got[n] - full[x4, x3, x2, x1])) < 1e-13


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 4, 2, 6)])
def test_gamma5_hermiticity_and_adjoint(dims):
    U = syn.gauge_field(dims, 0.3, 21)
    phi = syn.gaussian_spinor(dims, 22)
    psi = syn.gaussian_spinor(dims, 23)
    k = 0.12
    lhs = np.vdot(phi, wilson.gamma5(wilson.dirac(U, wilson.gamma5(psi), k)))
    rhs = np.vdot(wilson.dirac(U, phi, k), psi)
    assert abs(lhs - rhs) < 1e-10 * abs(rhs)
    # the dagger flag is the true adjoint
    lhs = np.vdot(phi, wilson.hop(U, psi))
    rhs = np.vdot(wilson.hop(U, phi, dagger=True), psi)
    assert abs(lhs - rhs) < 1e-10 * abs(rhs)
    # and equals gamma5 H gamma5
    a = wilson.hop(U, psi, dagger=True)
    b = wilson.gamma5(wilson.hop(U, wilson.gamma5(psi)))
    assert np.max(np.abs(a - b)) < 1e-12


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 4, 6, 4)])
def test_gauge_covariance(dims):
    U = syn.gauge_field(dims, 0.3, 31)
    psi = syn.gaussian_spinor(dims, 32)
    V = syn.volume(dims)
    Om = syn.random_su3(V, 33).reshape(syn.lattice_shape(dims) + (3, 3))
    Up, psip = wilson.gauge_transform(U, psi, Om)
    lhs = wilson.dirac(Up, psip, 0.124)
    rhs = wilson.colour_mul(Om, wilson.dirac(U, psi, 0.124))
    assert np.max(np.abs(lhs - rhs)) < 1e-12


def test_parity_split_and_kappa_zero():
    dims = (4, 4, 2, 6)
    U = syn.gauge_field(dims, 0.3, 41)
    psi = syn.gaussian_spinor(dims, 42)
    H = wilson.hop(U, psi)
    he = wilson.hop_parity(U, psi, 0)
    ho = wilson.hop_parity(U, psi, 1)
    assert np.max(np.abs(he + ho - H)) < 1e-12
    m0 = wilson.parity_mask(dims, 0)
    assert np.max(np.abs((1 - m0) * he)) == 0.0
    # a parity hop reads only the other parity
    assert np.max(np.abs(wilson.hop_parity(U, m0 * psi, 0))) == 0.0
    assert np.array_equal(wilson.dirac(U, psi, 0.0), psi)


def test_schur_equivalence_dense():
    """M_e = 1 - k^2 H_eo H_oe is the Schur complement of the dense D on even sites."""
    dims = (2, 4, 2, 4)
    U = syn.gauge_field(dims, 0.3, 51)
    k = 0.12
    D = wilson.dense_dirac(U, k)
    par = np.repeat(wilson.parity_field(dims).ravel(), 12)
    e = par == 0
    o = ~e
    S = D[np.ix_(e, e)] - D[np.ix_(e, o)] @ np.linalg.solve(D[np.ix_(o, o)], D[np.ix_(o, e)])
    psi = syn.gaussian_spinor(dims, 52) * wilson.parity_mask(dims, 0)
    got = wilson.flat(wilson.schur(U, psi, k, 0))[e]
    want = S @ wilson.flat(psi)[e]
    assert np.max(np.abs(got - want)) < 1e-12
    got_d = wilson.flat(wilson.schur(U, psi, k, 0, dagger=True))[e]
    assert np.max(np.abs(got_d - S.conj().T @ wilson.flat(psi)[e])) < 1e-12


def test_links_are_su3_and_compressible():
    U = syn.gauge_field((4, 4, 4, 4), 0.3, 61).reshape(-1, 3, 3)
    I = np.eye(3)
    assert np.max(np.abs(U @ np.conj(np.swapaxes(U, -1, -2)) - I)) < 1e-14
    assert np.max(np.abs(np.linalg.det(U) - 1)) < 1e-14
    r2 = np.conj(np.cross(U[:, 0], U[:, 1]))
    assert np.max(np.abs(r2 - U[:, 2])) == 0.0
    # near-unit: |U - 1| grows with eps
    d = np.abs(U - I).max()
    assert 0.05 < d < 2.0


def test_exactly_reduced_plane_wave_is_the_plane_wave():
    """plane_wave_n (integer momentum numbers, phase reduced exactly) equals
    exp(i p.x) u site by site, and D_W acts on it by the symbol to ~1e-15
    per site on a lattice where unreduced phases reach ~150."""
    dims = (8, 6, 4, 10)
    n = (3, 5, 1, 7)
    u = syn.gaussian_spinor((2, 2, 2, 2), 9)[0, 0, 0, 0]
    p = free_field.momentum_of(dims, n)
    assert np.allclose(p[3], 2 * np.pi * 7.5 / 10)
    a = free_field.plane_wave_n(dims, n, u)
    b = free_field.plane_wave(dims, p, u)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(u))
    U = syn.unit_gauge(dims)
    got = wilson.dirac(U, a, 0.124)
    want = free_field.plane_wave_n(dims, n, free_field.symbol(p, 0.124) @ u)
    assert np.max(np.abs(got - want)) <= 4e-15 * np.max(np.abs(want))
    # periodic time: integer n_4, no half shift
    pp = free_field.momentum_of(dims, n, tbc=+1)
    ap = free_field.plane_wave_n(dims, n, u, tbc=+1)
    assert np.max(np.abs(wilson.dirac(U, ap, 0.1, tbc=+1)
                         - free_field.plane_wave_n(dims, n, free_field.symbol(pp, 0.1) @ u, tbc=+1))) <= 4e-15 * 3
