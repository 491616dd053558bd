"""GPU parity of the parallel-transport convolution network and FGCR.

Forward with FP32 activations: relative difference <= 1e-5 against the FP64
oracle fed the same FP32-rounded links, inputs and weights (about 20
rounded FP32 operations per output component, well inside 1e-5).  With BF16
activations the oracle rounds the same stored activations to bfloat16; the
two sides may round a hidden value near a bfloat16 tie differently (the GPU
computes it in FP32, the oracle in FP64), so the bar is 2e-3.  Gradients
(FP32 arithmetic, FP64 site sums): <= 1e-4 relative.

Every forward comparison is also made site by site (largest real error of a
site over the site's largest expected |real|): 1e-4 with FP32 activations
(ten times the whole-field bar); 2^-5 with BF16 activations, since one
hidden value rounded to the neighbouring bfloat16 (2^-7 of it) reaches an
output site through 18 weighted terms of similar size; 2^-4 with FP16
products, whose 7 truncated operands give up to 7 * 2^-10 per term.  A
wrong entry of typical size at one site is off by ~1 on this scale.
"""
import numpy as np
import pytest
import torch

import paper_0710_2442_amd as wd
import synthetic as syn
from gpu_util import assert_close, from_field, rel_err, round_c64, storage_round, to_field
from oracle import ptc, solvers, wilson

pytestmark = pytest.mark.gpu

DIMS = (6, 4, 6, 10)


def _weights(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    z1 = rng.standard_normal((9, 2, 1, 4, 4, 2))
    z2 = rng.standard_normal((9, 1, 2, 4, 4, 2))
    W1 = scale * (z1[..., 0] + 1j * z1[..., 1])
    W2 = scale * (z2[..., 0] + 1j * z2[..., 1])
    # round once to complex64: both sides use the same weights
    return round_c64(W1), round_c64(W2)


def _bf16(a):
    """bfloat16 storage of activations, which the library keeps in its storage spin basis."""
    return storage_round(a, "bf16")


@pytest.mark.parametrize("act", ["f32", "bf16"])
def test_forward_matches_oracle(act):
    U = syn.gauge_field(DIMS, 0.3, 301)
    r = syn.gaussian_spinor(DIMS, 302)
    W1, W2 = _weights(303)
    g = wd.Gauge(U, DIMS, -1, "f32")
    n = wd.Ptc(g, wd.ptc_weights_to_flat(W1, W2), act)
    fr = to_field(g, r, "f32")
    fy = wd.wd_new_field(DIMS, "f32")
    wd.wd_ptc_apply(n, fr, fy)
    got = from_field(g, fy, "f32")
    Ur, rr = round_c64(U), storage_round(r, "f32")
    if act == "f32":
        want = ptc.network(Ur, rr, W1, W2)
        assert_close(got, want, l2=1e-5, site=1e-4, what="PTC forward, FP32 activations")
    else:
        want = ptc.network(Ur, rr, W1, W2, act_round=_bf16)
        assert_close(got, want, l2=2e-3, site=2.0 ** -5, what="PTC forward, BF16 activations")
    n.close()
    g.close()


@pytest.mark.parametrize("dims", [(6, 4, 6, 10), (8, 8, 8, 8), (6, 2, 2, 6)])
@pytest.mark.parametrize("scale", [1.0, 1e-7])
def test_even_application_matches_oracle(dims, scale):
    """[N(x_e, 0)]_e, as the even-odd solver applies the network, against the
    oracle's full network on a field that is zero on odd sites.

    FP32 products (flags 0): the bar of the BF16 forward test (2e-3).  FP16
    products with FP32 sums: every operand of a product chain (input, link,
    transported spinor, weight, mixed spinor, link, weight: 7) is rounded
    toward zero to 11 significant bits, a relative error below 2^-10 each
    and biased one way, so up to 7 * 2^-10 ~ 7e-3 on a component; bar 1e-2.
    A tiny input (1e-7) checks the scaling to unit RMS: without it the FP16
    operands would underflow.  BF16 operands on the matrix cores: every
    operand of a chain (input, link rows, rebuilt link row, transported
    spinor, weight, hidden channel, weight, mixed spinor, link) is rounded to
    nearest at 8 significant bits, below 2^-9 relative each, so up to
    9 * 2^-9 ~ 1.8e-2 on a component; bar 2e-2, per site 2^-3.  BF16 keeps
    FP32's exponent range, so the tiny input needs no scaling there."""
    U = syn.gauge_field(dims, 0.3, 305)
    x = syn.gaussian_spinor(dims, 306) * scale
    W1, W2 = _weights(307)
    g = wd.Gauge(U, dims, -1, "f32")
    n = wd.Ptc(g, wd.ptc_weights_to_flat(W1, W2), "bf16")
    fx = to_field(g, x, "f32", wd.WD_EVEN)
    even = wilson.parity_mask(dims, 0)
    xe = storage_round(x * even, "f32")
    want = ptc.network(round_c64(U), xe, W1, W2, act_round=_bf16) * even
    for flags, bar, sbar in ((0, 2e-3, 2.0 ** -5), (wd.WD_PTC_FP16_PRODUCTS, 1e-2, 2.0 ** -4),
                             (wd.WD_PTC_BF16_MFMA, 2e-2, 2.0 ** -3)):
        for pout in ("f32", "bf16"):
            fy = wd.wd_new_field(dims, pout, 1, wd.WD_EVEN)
            wd.wd_ptc_apply_even(n, fx, "f32", fy, pout, flags)
            got = from_field(g, fy, pout, wd.WD_EVEN)
            extra = 2.0 ** -8 if pout == "bf16" else 0.0  # the stored output's own rounding
            assert_close(got, want, l2=bar + extra, site=sbar + extra,
                         what=f"PTC even {dims} x{scale} flags={flags} out={pout}")
    with pytest.raises(wd.WdError):  # FP16 products need BF16 activations
        n32 = wd.Ptc(g, wd.ptc_weights_to_flat(W1, W2), "f32")
        try:
            fy = wd.wd_new_field(dims, "f32", 1, wd.WD_EVEN)
            wd.wd_ptc_apply_even(n32, fx, "f32", fy, "f32", wd.WD_PTC_FP16_PRODUCTS)
        finally:
            n32.close()
    n.close()
    g.close()


def test_gauge_equivariance_on_gpu():
    U = syn.gauge_field(DIMS, 0.3, 311)
    r = syn.gaussian_spinor(DIMS, 312)
    W1, W2 = _weights(313)
    Om = syn.random_su3(syn.volume(DIMS), 314).reshape(syn.lattice_shape(DIMS) + (3, 3))
    Up, rp = wilson.gauge_transform(U, r, Om)
    outs = []
    for (UU, rr) in ((U, r), (Up, rp)):
        g = wd.Gauge(UU, DIMS, -1, "f32")
        n = wd.Ptc(g, wd.ptc_weights_to_flat(W1, W2), "f32")
        fy = wd.wd_new_field(DIMS, "f32")
        wd.wd_ptc_apply(n, to_field(g, rr, "f32"), fy)
        outs.append(from_field(g, fy, "f32"))
        n.close()
        g.close()
    assert_close(outs[1], wilson.colour_mul(Om, outs[0]), l2=1e-5, site=1e-4, what="PTC equivariance")


def _pairs(B, seed):
    rs = syn.gaussian_spinor(DIMS, seed, nrhs=B)
    es = syn.gaussian_spinor(DIMS, seed + 1, nrhs=B)
    return rs, es


def test_loss_and_gradients_match_oracle():
    U = syn.gauge_field(DIMS, 0.3, 321)
    W1, W2 = _weights(322, scale=0.2)
    rs, es = _pairs(2, 323)
    g = wd.Gauge(U, DIMS, -1, "f32")
    n = wd.Ptc(g, wd.ptc_weights_to_flat(W1, W2), "f32")
    fr = torch.cat([to_field(g, rs[b], "f32") for b in range(2)])
    fe = torch.cat([to_field(g, es[b], "f32") for b in range(2)])
    loss, grad = wd.wd_ptc_loss_grad(n, fr, fe, 2)
    Ur = round_c64(U)
    L, g1, g2 = ptc.loss_and_grads(Ur, W1, W2, [storage_round(x, "f32") for x in rs],
                                   [storage_round(x, "f32") for x in es])
    assert abs(loss - L) <= 1e-5 * L
    G1, G2 = wd.ptc_flat_to_weights(grad)
    want = np.concatenate([g1.ravel(), g2.ravel()])
    got = np.concatenate([G1.ravel(), G2.ravel()])
    assert rel_err(got, want) <= 1e-4, rel_err(got, want)
    # deterministic: a second evaluation is bit for bit the same
    loss2, grad2 = wd.wd_ptc_loss_grad(n, fr, fe, 2)
    assert loss2 == loss and np.array_equal(grad, grad2)
    n.close()
    g.close()


def test_adam_steps_follow_oracle_and_reduce_loss():
    U = syn.gauge_field(DIMS, 0.3, 331)
    W1, W2 = ptc.init_weights(332)
    W1, W2 = round_c64(W1), round_c64(W2)
    rs, es = _pairs(2, 333)
    g = wd.Gauge(U, DIMS, -1, "f32")
    flat0 = wd.ptc_weights_to_flat(W1, W2)
    n = wd.Ptc(g, flat0, "f32")
    fr = torch.cat([to_field(g, rs[b], "f32") for b in range(2)])
    fe = torch.cat([to_field(g, es[b], "f32") for b in range(2)])
    lr = 1e-3
    l0 = wd.wd_ptc_train_step(n, fr, fe, 2, lr)
    W_gpu = wd.wd_ptc_get_weights(n)
    # oracle: one Adam step from the same weights with the oracle's gradients
    Ur = round_c64(U)
    L, g1, g2 = ptc.loss_and_grads(Ur, W1, W2, [storage_round(x, "f32") for x in rs],
                                   [storage_round(x, "f32") for x in es])
    gflat = np.concatenate([g1.ravel(), g2.ravel()])
    w = np.concatenate([W1.ravel(), W2.ravel()])
    w1, _, _ = ptc.adam_step(w, gflat, np.zeros((2, 576)), np.zeros((2, 576)), 1, lr=lr)
    got = W_gpu.view(np.complex64).astype(np.complex128)
    gmax = np.max(np.abs(np.concatenate([gflat.real, gflat.imag])))
    sel_re = np.abs(gflat.real) > 1e-3 * gmax
    sel_im = np.abs(gflat.imag) > 1e-3 * gmax
    assert np.max(np.abs((got - w1).real[sel_re])) <= 1e-2 * lr
    assert np.max(np.abs((got - w1).imag[sel_im])) <= 1e-2 * lr
    assert abs(l0 - L) <= 1e-5 * L
    losses = [l0] + [wd.wd_ptc_train_step(n, fr, fe, 2, lr) for _ in range(20)]
    assert losses[-1] < 0.95 * losses[0]
    n.close()
    g.close()


# ------------------------------------------------------------------ FGCR
def _fgcr(dims, kappa, net_flat=None, act="bf16", m=12, seed=341, solver=None, **kw):
    U = syn.gauge_field(dims, 0.3, seed)
    b = syn.gaussian_spinor(dims, seed + 1)
    g = wd.Gauge(U, dims, -1, "f64")
    n = wd.Ptc(g, net_flat, act) if net_flat is not None else None
    fb = to_field(g, b)
    fx = wd.wd_new_field(dims, "f64")
    p = wd.wd_solve_params_default(solver=wd.WD_SOLVER_FGCR if solver is None else solver, fgcr_m=m, precond=n,
                                   **kw)
    rc, info = wd.wd_solve(g, fb, fx, kappa, 1e-10, p)
    x = from_field(g, fx)
    if n is not None:
        n.close()
    g.close()
    return U, b, x, rc, info


def test_fgcr_identity_matches_oracle_gcr():
    dims, kappa = (8, 8, 8, 8), 0.124
    U, b, x, rc, info = _fgcr(dims, kappa, None, m=64)
    assert rc == 0 and info["fallback_used"] == 0
    assert solvers.true_residual(U, b, x, kappa) <= 1e-10
    Dop = lambda v: wilson.dirac(U, v, kappa)
    xo, it_o, fb, _ = solvers.fgcr(Dop, lambda r: r, b, 1e-10, m=64, stagnation=1000)
    assert abs(info["iters"] - it_o) <= 2, (info["iters"], it_o)
    assert rel_err(x, xo) <= 1e-7


@pytest.mark.parametrize("act", ["f32", "bf16"])
def test_fgcr_with_network_converges(act):
    dims, kappa = (8, 8, 8, 8), 0.124
    W1, W2 = ptc.init_weights(351)
    U, b, x, rc, info = _fgcr(dims, kappa, wd.ptc_weights_to_flat(W1, W2), act)
    assert rc == 0 and info["fallback_used"] == 0
    assert solvers.true_residual(U, b, x, kappa) <= 1e-10


@pytest.mark.parametrize("bad", ["zero", "nan"])
def test_fgcr_falls_back_to_cg(bad):
    dims, kappa = (8, 8, 8, 8), 0.124
    flat = np.zeros(1152, np.float32) if bad == "zero" else np.full(1152, np.nan, np.float32)
    if bad == "nan":
        # the library refuses non-finite weights at creation; corrupt them afterwards
        U = syn.gauge_field(dims, 0.3, 361)
        b = syn.gaussian_spinor(dims, 362)
        g = wd.Gauge(U, dims, -1, "f64")
        n = wd.Ptc(g, np.zeros(1152, np.float32), "f32")
        with pytest.raises(wd.WdError):
            wd.Ptc(g, flat, "f32")
        big = np.full(1152, 3e38, np.float32)  # overflows to inf inside the network
        wd.wd_ptc_set_weights(n, big)
        fb = to_field(g, b)
        fx = wd.wd_new_field(dims, "f64")
        p = wd.wd_solve_params_default(solver=wd.WD_SOLVER_FGCR, precond=n)
        rc, info = wd.wd_solve(g, fb, fx, kappa, 1e-10, p)
        x = from_field(g, fx)
        n.close()
        g.close()
    else:
        U, b, x, rc, info = _fgcr(dims, kappa, flat, "f32", seed=361)
    assert rc == 0 and info["fallback_used"] == 1
    assert solvers.true_residual(U, b, x, kappa) <= 1e-10


# ------------------------------------------------- mixed-precision even-odd FGCR
@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (6, 4, 6, 10)])
@pytest.mark.parametrize("net", [None, "f32", "bf16"])
@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_defect_fgcr_reaches_fp64_residual(dims, net, store):
    """FP32-arithmetic eo-FGCR (inner vectors stored in FP32 or BF16) inside
    FP64 defect correction: the oracle's own D_W must see a true residual
    <= 1e-10, the reported residual must agree, and the solution must agree
    with the oracle's FP64 eo-CGLS solution."""
    kappa = 0.124
    flat = None if net is None else wd.ptc_weights_to_flat(*ptc.init_weights(353))
    U, b, x, rc, info = _fgcr(dims, kappa, flat, net or "bf16", m=8, solver=wd.WD_SOLVER_DEFECT_FGCR,
                              inner_tol=1e-3 if store == "f32" else 1e-2, inner_prec=store)
    assert rc == 0 and info["fallback_used"] == 0, info
    r = solvers.true_residual(U, b, x, kappa)
    assert r <= 1e-10
    assert abs(r - info["true_rel_resid"]) <= 1e-3 * 1e-10 + 1e-15
    assert info["outer_iters"] >= 2  # FP32 inner: at least one correction
    xo, _, _ = solvers.solve_eo_cgls(U, b, kappa, 1e-12)
    assert rel_err(x, xo) <= 1e-7


@pytest.mark.parametrize("m", [1, 4, 16])
@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_defect_fgcr_restart_lengths(m, store):
    U, b, x, rc, info = _fgcr((8, 8, 8, 8), 0.124, None, m=m, solver=wd.WD_SOLVER_DEFECT_FGCR, inner_prec=store)
    assert rc == 0 and info["fallback_used"] == 0
    assert solvers.true_residual(U, b, x, 0.124) <= 1e-10


@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_defect_fgcr_is_deterministic(store):
    a = _fgcr((8, 8, 8, 8), 0.124, wd.ptc_weights_to_flat(*ptc.init_weights(354)), "bf16", m=8,
              solver=wd.WD_SOLVER_DEFECT_FGCR, inner_prec=store)
    b = _fgcr((8, 8, 8, 8), 0.124, wd.ptc_weights_to_flat(*ptc.init_weights(354)), "bf16", m=8,
              solver=wd.WD_SOLVER_DEFECT_FGCR, inner_prec=store)
    assert a[4]["iters"] == b[4]["iters"] and np.array_equal(a[2], b[2])


def test_defect_fgcr_rejects_bad_parameters():
    dims = (4, 4, 4, 4)
    g = wd.Gauge(syn.gauge_field(dims, 0.3, 355), dims, -1, "f64")
    fb = to_field(g, syn.gaussian_spinor(dims, 356))
    fx = wd.wd_new_field(dims, "f64")
    for kw in (dict(fgcr_m=17), dict(inner_prec="f16"), dict(inner_prec="f64")):
        p = wd.wd_solve_params_default(solver=wd.WD_SOLVER_DEFECT_FGCR, **kw)
        with pytest.raises(wd.WdError):
            wd.wd_solve(g, fb, fx, 0.124, 1e-10, p)
    g.close()


def test_defect_fgcr_falls_back_to_cg_on_overflow():
    dims, kappa = (8, 8, 8, 8), 0.124
    U = syn.gauge_field(dims, 0.3, 363)
    b = syn.gaussian_spinor(dims, 364)
    g = wd.Gauge(U, dims, -1, "f64")
    n = wd.Ptc(g, np.zeros(1152, np.float32), "f32")
    wd.wd_ptc_set_weights(n, np.full(1152, 3e38, np.float32))  # overflows to inf inside the network
    fb = to_field(g, b)
    fx = wd.wd_new_field(dims, "f64")
    p = wd.wd_solve_params_default(solver=wd.WD_SOLVER_DEFECT_FGCR, precond=n)
    rc, info = wd.wd_solve(g, fb, fx, kappa, 1e-10, p)
    x = from_field(g, fx)
    n.close()
    g.close()
    assert rc == 0 and info["fallback_used"] == 1
    assert solvers.true_residual(U, b, x, kappa) <= 1e-10
