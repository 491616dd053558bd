"""Gauge-covariant parallel-transport convolution (PTC) network, FP64.

Test infrastructure only.  The paper has no network; this is the reading used
for the learned right preconditioner of the flexible GCR solver.

A layer maps C_in spinor fields psi_c to C_out fields
    y_{c'}(x) = sum_c sum_h W^{(h)}_{c'c} (T_h psi_c)(x)
over the nine hops h = 0 (T_0 = 1), h = 1..4 (T_{+mu}) and h = 5..8
(T_{-mu}), mu = x1..x4:
    (T_{+mu} psi)(x) = U_{x,mu} psi(x+mu)
    (T_{-mu} psi)(x) = U^dag_{x-mu,mu} psi(x-mu)
with the same time-boundary factor as Eq. 3.  W^{(h)}_{c'c} is a complex
4x4 matrix acting on spin only, so each layer commutes with gauge
transformations psi -> Omega psi.  No bias and no nonlinearity.

Network: r -> layer1 (1 -> 2 channels) -> layer2 (2 -> 1 channel); weights
shaped (9, C_out, C_in, 4, 4): 9*2*16 + 9*2*16 = 576 complex parameters.
"""
from __future__ import annotations

import numpy as np

from . import wilson
from .wilson import colour_mul, colour_mul_dag, shift_backward, shift_forward

NHOP = 9


def transport(U, psi, h, tbc=-1):
    """T_h psi for h in 0..8 (see module docstring)."""
    if h == 0:
        return psi.copy()
    if h <= 4:
        mu = h - 1
        return colour_mul(U[..., mu, :, :], shift_forward(psi, mu, tbc))
    mu = h - 5
    return colour_mul_dag(shift_backward(U[..., mu, :, :], mu, 1), shift_backward(psi, mu, tbc))


def adjoint_hop(h):
    """Index of T_h^dag:  T_0^dag = T_0, T_{+mu}^dag = T_{-mu}, T_{-mu}^dag = T_{+mu}."""
    if h == 0:
        return 0
    return h + 4 if h <= 4 else h - 4


def layer(U, psi, W, tbc=-1):
    """One PTC layer.  psi: (C_in, L4,L3,L2,L1,4,3); W: (9, C_out, C_in, 4, 4)."""
    nh, cout, cin = W.shape[:3]
    y = np.zeros((cout,) + psi.shape[1:], dtype=np.complex128)
    for c in range(cin):
        for h in range(nh):
            t = transport(U, psi[c], h, tbc)
            for co in range(cout):
                y[co] += wilson.spin_mul(W[h, co, c], t)
    return y


def layer_backward(U, psi, W, gy, tbc=-1):
    """Gradients of a real loss through one layer.

    ``gy`` = dL/dRe(y) + i dL/dIm(y).  Returns (g_psi, g_W) in the same
    convention:
      g_psi_c = sum_{c'} sum_h T_h^dag ( W^{(h)dag}_{c'c} gy_{c'} )
      g_W^{(h)}_{c'c}[s',s] = sum_x sum_colour gy_{c'}(x)[s',a] conj((T_h psi_c)(x)[s,a])
    """
    nh, cout, cin = W.shape[:3]
    gpsi = np.zeros_like(psi, dtype=np.complex128)
    gW = np.zeros_like(W, dtype=np.complex128)
    for c in range(cin):
        for h in range(nh):
            t = transport(U, psi[c], h, tbc)
            for co in range(cout):
                gW[h, co, c] = np.einsum("nsa,nta->st", gy[co].reshape(-1, 4, 3),
                                          np.conj(t).reshape(-1, 4, 3))
                v = wilson.spin_mul(np.conj(W[h, co, c]).T, gy[co])
                gpsi[c] += transport(U, v, adjoint_hop(h), tbc)
    return gpsi, gW


def network(U, r, W1, W2, tbc=-1, act_round=None):
    """N(r) for a single-channel field r (L4,L3,L2,L1,4,3).

    ``act_round`` (optional) rounds the stored activations (the network input
    and the hidden layer) like a reduced-precision store would.
    """
    x0 = r[None]
    if act_round is not None:
        x0 = act_round(x0)
    y1 = layer(U, x0, W1, tbc)
    if act_round is not None:
        y1 = act_round(y1)
    y2 = layer(U, y1, W2, tbc)
    return y2[0]


def network_backward(U, r, W1, W2, g_out, tbc=-1):
    """Returns (g_r, g_W1, g_W2) for the FP64 network (no activation rounding)."""
    x0 = r[None]
    y1 = layer(U, x0, W1, tbc)
    g_y1, gW2 = layer_backward(U, y1, W2, g_out[None], tbc)
    g_x0, gW1 = layer_backward(U, x0, W1, g_y1, tbc)
    return g_x0[0], gW1, gW2


def loss(U, W1, W2, rs, es, tbc=-1):
    """Mean over the batch of |N(r_b) - e_b|^2 (pairs already normalised)."""
    tot = 0.0
    for r, e in zip(rs, es):
        d = network(U, r, W1, W2, tbc) - e
        tot += float(np.vdot(d.ravel(), d.ravel()).real)
    return tot / len(rs)


def loss_and_grads(U, W1, W2, rs, es, tbc=-1):
    B = len(rs)
    gW1 = np.zeros_like(W1)
    gW2 = np.zeros_like(W2)
    tot = 0.0
    for r, e in zip(rs, es):
        d = network(U, r, W1, W2, tbc) - e
        tot += float(np.vdot(d.ravel(), d.ravel()).real)
        _, g1, g2 = network_backward(U, r, W1, W2, (2.0 / B) * d, tbc)
        gW1 += g1
        gW2 += g2
    return tot / B, gW1, gW2


def init_weights(seed, cin_cout=((1, 2), (2, 1)), scale=1e-2):
    """Near-identity init: W^{(0)} = I/sqrt(2) in both layers, other hops N(0, scale^2)."""
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    Ws = []
    for cin, cout in cin_cout:
        z = rng.standard_normal((NHOP, cout, cin, 4, 4, 2))
        W = scale * (z[..., 0] + 1j * z[..., 1]) / np.sqrt(2.0)
        for co in range(cout):
            for c in range(cin):
                W[0, co, c] = np.eye(4) / np.sqrt(2.0)
        Ws.append(W)
    return Ws


def adam_step(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma & Ba) on the real and imaginary parts separately.  Returns (w, m, v)."""
    gr = np.stack([g.real, g.imag])
    m = b1 * m + (1 - b1) * gr
    v = b2 * v + (1 - b2) * gr * gr
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    step = lr * mh / (np.sqrt(vh) + eps)
    w = w - (step[0] + 1j * step[1])
    return w, m, v
