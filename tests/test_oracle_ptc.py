"""Pins of the oracle's parallel-transport convolution network."""
import numpy as np
import pytest

import synthetic as syn
from oracle import free_field, ptc, wilson


def _rand_w(rng, cout, cin, scale=0.3):
    z = rng.standard_normal((9, cout, cin, 4, 4, 2))
    return scale * (z[..., 0] + 1j * z[..., 1])


def test_parameter_count():
    W1, W2 = ptc.init_weights(0)
    assert W1.shape == (9, 2, 1, 4, 4) and W2.shape == (9, 1, 2, 4, 4)
    assert W1.size + W2.size == 576


def test_adjoint_transport():
    dims = (4, 2, 4, 6)
    U = syn.gauge_field(dims, 0.4, 201)
    a = syn.gaussian_spinor(dims, 202)
    b = syn.gaussian_spinor(dims, 203)
    for h in range(9):
        lhs = np.vdot(a, ptc.transport(U, b, h))
        rhs = np.vdot(ptc.transport(U, a, ptc.adjoint_hop(h)), b)
        assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_gauge_equivariance():
    dims = (4, 4, 2, 4)
    rng = np.random.default_rng(3)
    U = syn.gauge_field(dims, 0.3, 211)
    r = syn.gaussian_spinor(dims, 212)
    W1, W2 = _rand_w(rng, 2, 1), _rand_w(rng, 1, 2)
    Om = syn.random_su3(syn.volume(dims), 213).reshape(syn.lattice_shape(dims) + (3, 3))
    Up, rp = wilson.gauge_transform(U, r, Om)
    lhs = ptc.network(Up, rp, W1, W2)
    rhs = wilson.colour_mul(Om, ptc.network(U, r, W1, W2))
    assert np.max(np.abs(lhs - rhs)) < 1e-12


def test_identity_hop_only_is_sitewise_spin_matrix():
    dims = (2, 4, 2, 4)
    rng = np.random.default_rng(4)
    U = syn.gauge_field(dims, 0.3, 221)
    r = syn.gaussian_spinor(dims, 222)
    W1 = np.zeros((9, 2, 1, 4, 4), complex)
    W2 = np.zeros((9, 1, 2, 4, 4), complex)
    W1[0] = _rand_w(rng, 2, 1)[0]
    W2[0] = _rand_w(rng, 1, 2)[0]
    M = W2[0, 0, 0] @ W1[0, 0, 0] + W2[0, 0, 1] @ W1[0, 1, 0]
    got = ptc.network(U, r, W1, W2)
    assert np.max(np.abs(got - wilson.spin_mul(M, r))) < 1e-13


def test_unit_links_plane_wave_symbol():
    """U = 1: a layer multiplies e^{ipx}u by W0 + sum_mu (W+mu e^{ip_mu} + W-mu e^{-ip_mu})."""
    dims = (4, 2, 4, 6)
    rng = np.random.default_rng(5)
    U = syn.unit_gauge(dims)
    W = _rand_w(rng, 1, 1)
    p = [2 * np.pi * 1 / 4, 2 * np.pi * 1 / 2, 2 * np.pi * 3 / 4, 2 * np.pi * (2 + 0.5) / 6]
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    psi = free_field.plane_wave(dims, p, u)
    got = ptc.layer(U, psi[None], W)[0]
    S = W[0, 0, 0].copy()
    for mu in range(4):
        S = S + W[1 + mu, 0, 0] * np.exp(1j * p[mu]) + W[5 + mu, 0, 0] * np.exp(-1j * p[mu])
    want = free_field.plane_wave(dims, p, S @ u)
    assert np.max(np.abs(got - want)) < 1e-12


def test_backward_matches_finite_differences():
    dims = (2, 2, 2, 4)
    rng = np.random.default_rng(6)
    U = syn.gauge_field(dims, 0.3, 231)
    rs = [syn.gaussian_spinor(dims, 232), syn.gaussian_spinor(dims, 233)]
    es = [syn.gaussian_spinor(dims, 234), syn.gaussian_spinor(dims, 235)]
    W1, W2 = _rand_w(rng, 2, 1), _rand_w(rng, 1, 2)
    L, g1, g2 = ptc.loss_and_grads(U, W1, W2, rs, es)
    assert abs(L - ptc.loss(U, W1, W2, rs, es)) < 1e-12 * L
    h = 1e-6
    for (W, g, which) in ((W1, g1, 0), (W2, g2, 1)):
        for _ in range(12):
            idx = tuple(rng.integers(0, s) for s in W.shape)
            for part, unit in (("re", 1.0), ("im", 1j)):
                Wp = W.copy(); Wp[idx] += h * unit
                Wm = W.copy(); Wm[idx] -= h * unit
                args_p = (Wp, W2) if which == 0 else (W1, Wp)
                args_m = (Wm, W2) if which == 0 else (W1, Wm)
                fd = (ptc.loss(U, *args_p, rs, es) - ptc.loss(U, *args_m, rs, es)) / (2 * h)
                an = g[idx].real if part == "re" else g[idx].imag
                assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (which, idx, part, fd, an)
    # input gradient of a single sample
    r, e = rs[0], es[0]
    d = ptc.network(U, r, W1, W2) - e
    gr, _, _ = ptc.network_backward(U, r, W1, W2, 2.0 * d)
    f = lambda rr: float(np.vdot(ptc.network(U, rr, W1, W2) - e, ptc.network(U, rr, W1, W2) - e).real)
    for _ in range(6):
        idx = tuple(rng.integers(0, s) for s in r.shape)
        for unit in (1.0, 1j):
            rp = r.copy(); rp[idx] += h * unit
            rm = r.copy(); rm[idx] -= h * unit
            fd = (f(rp) - f(rm)) / (2 * h)
            an = gr[idx].real if unit == 1.0 else gr[idx].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def test_adam_first_step_is_lr_sign():
    """Adam's first update has magnitude lr in every coordinate with nonzero gradient."""
    rng = np.random.default_rng(8)
    w = rng.standard_normal(10) + 1j * rng.standard_normal(10)
    g = rng.standard_normal(10) + 1j * rng.standard_normal(10)
    m = np.zeros((2, 10)); v = np.zeros((2, 10))
    w2, m, v = ptc.adam_step(w, g, m, v, 1, lr=1e-3, eps=0.0)
    d = w2 - w
    assert np.allclose(d.real, -1e-3 * np.sign(g.real))
    assert np.allclose(d.imag, -1e-3 * np.sign(g.imag))


def test_adam_constant_gradient_steps_by_lr_at_every_step():
    """Kingma & Ba's bias corrections make m_hat = g and v_hat = g^2 exactly
    when the gradient never changes, so every step (t = 1, 2, 3, ...) moves
    each coordinate by lr * g / (|g| + eps).  Without the corrections step 2
    would be (0.19 / sqrt(0.001999)) lr = 4.25 lr."""
    g = np.array([0.5 - 2.0j, -3.0 + 0.25j, 1e-3 + 7.0j])
    w = np.zeros(3, dtype=np.complex128)
    m = np.zeros((2, 3)); v = np.zeros((2, 3))
    lr, eps = 1e-2, 1e-8
    want_re = lr * g.real / (np.abs(g.real) + eps)
    want_im = lr * g.imag / (np.abs(g.imag) + eps)
    for t in (1, 2, 3, 4):
        w2, m, v = ptc.adam_step(w, g, m, v, t, lr=lr, eps=eps)
        d = w - w2
        assert np.allclose(d.real, want_re, rtol=1e-12, atol=0), t
        assert np.allclose(d.imag, want_im, rtol=1e-12, atol=0), t
        w = w2


def test_adam_three_steps_hand_computed():
    """Gradients 1, 2, -1 on one real coordinate (and 0 on its imaginary
    part), beta = (0.9, 0.999), eps negligible (1e-300), worked out by hand from the
    definitions m_t = b1 m + (1 - b1) g, v_t = b2 v + (1 - b2) g^2,
    step = lr (m_t / (1 - b1^t)) / sqrt(v_t / (1 - b2^t)):
      t=1: m = 0.1,  v = 0.001,    step = lr
      t=2: m = 0.29, v = 0.004999, m_hat = 0.29/0.19, v_hat = 0.004999/0.001999
      t=3: m = 0.161, v = 0.005994001, m_hat = 0.161/0.271,
           v_hat = 0.005994001/0.002997001
    A swapped beta pair, a missing or squared correction, or a sign slip
    changes the second or third step by more than 1%."""
    lr = 1.0
    w = np.zeros(1, dtype=np.complex128)
    m = np.zeros((2, 1)); v = np.zeros((2, 1))
    steps = []
    for t, gv in enumerate((1.0, 2.0, -1.0), start=1):
        w2, m, v = ptc.adam_step(w, np.array([gv + 0j]), m, v, t, lr=lr, eps=1e-300)
        steps.append(float((w - w2).real[0]))
        assert (w2 - w).imag[0] == 0.0
        w = w2
    want = [1.0,
            (0.29 / 0.19) / np.sqrt(0.004999 / 0.001999),
            (0.161 / 0.271) / np.sqrt(0.005994001 / 0.002997001)]
    assert np.allclose(steps, want, rtol=1e-12, atol=0), (steps, want)
    assert abs(steps[1] - 0.96518) < 1e-4 and abs(steps[2] - 0.42009) < 1e-4
