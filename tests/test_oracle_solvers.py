"""Pins of the oracle's solvers: dense direct solves, the free-field FFT
solution, the Schur split, low-precision emulation and FGCR."""
import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import free_field, solvers, wilson


def _dense_solution(U, b, kappa):
    D = wilson.dense_dirac(U, kappa)
    x = np.linalg.solve(D, wilson.flat(b))
    return wilson.unflat(x, wilson.dims_of(b)), D


@pytest.mark.parametrize("dims", [(2, 4, 2, 6), (4, 4, 4, 4)])
def test_cgls_full_matches_dense(dims):
    U = syn.gauge_field(dims, 0.3, 101)
    b = syn.gaussian_spinor(dims, 102)
    k = 0.12
    xs, D = _dense_solution(U, b, k)
    x, it, hist = solvers.solve_cgls_full(U, b, k, 1e-10)
    assert solvers.true_residual(U, b, x, k) <= 1.5e-10
    cond = np.linalg.cond(D)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= cond * 2e-10
    assert hist[-1] <= 1e-10 and it > 5


@pytest.mark.parametrize("dims", [(2, 4, 2, 6), (4, 4, 4, 4)])
def test_eo_cgls_matches_dense(dims):
    U = syn.gauge_field(dims, 0.3, 111)
    b = syn.gaussian_spinor(dims, 112)
    k = 0.124
    xs, D = _dense_solution(U, b, k)
    x, it, hist = solvers.solve_eo_cgls(U, b, k, 1e-10)
    rel = solvers.true_residual(U, b, x, k)
    assert rel <= 2e-10
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= np.linalg.cond(D) * 3e-10
    # the odd-site residual vanishes by construction
    r = b - wilson.dirac(U, x, k)
    assert np.linalg.norm(wilson.parity_mask(dims, 1) * r) < 1e-12 * np.linalg.norm(b)


def test_kappa_zero_solve_is_identity():
    dims = (4, 4, 4, 4)
    U = syn.gauge_field(dims, 0.3, 121)
    b = syn.gaussian_spinor(dims, 122)
    x, it, _ = solvers.solve_eo_cgls(U, b, 0.0, 1e-10)
    assert np.max(np.abs(x - b)) < 1e-15
    assert it <= 1


@pytest.mark.parametrize("dims", [(2, 4, 2, 6), (4, 4, 4, 4)])
def test_fft_free_solution_matches_dense(dims):
    U = syn.unit_gauge(dims)
    b = syn.gaussian_spinor(dims, 131)
    k = 0.124
    xs, _ = _dense_solution(U, b, k)
    x = free_field.solve(b, k)
    assert np.max(np.abs(x - xs)) < 1e-10 * np.max(np.abs(xs))


def test_fft_free_solution_residual_8x4():
    dims = (8, 8, 8, 8)
    U = syn.unit_gauge(dims)
    b = syn.gaussian_spinor(dims, 141)
    x = free_field.solve(b, 0.124)
    assert solvers.true_residual(U, b, x, 0.124) < 1e-13


def test_free_condition_number():
    lo, hi = free_field.lambda_min_normal((32, 32, 32, 64), 0.124)
    # lambda_min(D^dag D) of the near-critical free operator on 32^3x64
    assert 1e-4 < lo < 1e-3
    assert 1e4 < hi / lo < 3e4
    lo8, hi8 = free_field.lambda_min_normal((8, 8, 8, 8), 0.12)
    assert 200 < hi8 / lo8 < 500


def test_round_bf16_matches_library():
    rng = np.random.default_rng(5)
    a = np.concatenate([
        rng.standard_normal(10000).astype(np.float32) * 10.0 ** rng.integers(-20, 20, 10000),
        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.5 - 2 ** -9, 0.0, 65504.0], dtype=np.float32),
    ]).astype(np.float32)
    want = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(solvers.round_bf16(a), want)


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_defect_correction_reaches_fp64_tolerance(storage):
    dims = (4, 4, 4, 4)
    U = syn.gauge_field(dims, 0.3, 151)
    b = syn.gaussian_spinor(dims, 152)
    k = 0.124
    xs, D = _dense_solution(U, b, k)
    x, outer, inner = solvers.solve_defect_correction(U, b, k, 1e-10, inner_tol=1e-2, storage=storage)
    assert solvers.true_residual(U, b, x, k) <= 1e-10
    assert outer >= 2  # the inner precision alone cannot reach 1e-10
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= np.linalg.cond(D) * 1e-10


def test_fgcr_identity_is_gcr_and_exact_preconditioner():
    dims = (2, 2, 2, 2)
    U = syn.gauge_field(dims, 0.3, 161)
    b = syn.gaussian_spinor(dims, 162)
    k = 0.124
    xs, D = _dense_solution(U, b, k)
    Dop = lambda v: wilson.dirac(U, v, k)
    # N = 1: plain GCR, converges in at most n = 192 directions
    x, it, fb, hist = solvers.fgcr(Dop, lambda r: r, b, 1e-10, m=200, stagnation=1000)
    assert not fb and it <= 192
    assert solvers.true_residual(U, b, x, k) <= 1e-10
    # residual norms of GCR never increase
    assert all(h2 <= h1 * (1 + 1e-12) for h1, h2 in zip(hist, hist[1:]))
    # N = D^{-1}: one direction suffices
    Dinv = np.linalg.inv(D)
    Nexact = lambda r: wilson.unflat(Dinv @ wilson.flat(r), dims)
    x, it, fb, _ = solvers.fgcr(Dop, Nexact, b, 1e-10, m=8)
    assert it == 1 and not fb
    assert np.max(np.abs(x - xs)) < 1e-10 * np.max(np.abs(xs))


def test_fgcr_falls_back_on_bad_preconditioner():
    dims = (2, 4, 2, 4)
    U = syn.gauge_field(dims, 0.3, 171)
    b = syn.gaussian_spinor(dims, 172)
    k = 0.12
    Dop = lambda v: wilson.dirac(U, v, k)

    def fallback(x, r):
        e, _, _ = solvers.solve_cgls_full(U, r, k, 1e-11 * np.linalg.norm(b) / np.linalg.norm(r))
        return e

    nan_net = lambda r: np.full_like(r, np.nan)
    x, it, fb, _ = solvers.fgcr(Dop, nan_net, b, 1e-10, cg_fallback=fallback)
    assert fb and it == 1
    assert solvers.true_residual(U, b, x, k) <= 1e-10
    zero_net = lambda r: np.zeros_like(r)
    x, it, fb, _ = solvers.fgcr(Dop, zero_net, b, 1e-10, cg_fallback=fallback)
    assert fb
    assert solvers.true_residual(U, b, x, k) <= 1e-10


def test_round_storage_f16_hand_values():
    """FP16 storage with a per-site scale (reading A11): the site's largest
    |real| m is kept exactly, every real is divided by m, rounded to IEEE half
    (to nearest, ties to even, with subnormals) and multiplied back.  One site
    with m = 2 (so the scaling is exact), worked out by hand:
      x/m = 1 - 2^-12   : halfway between 1 - 2^-11 (odd) and 1 (even) -> 1
      x/m = 1 - 3*2^-12 : halfway between 1 - 2^-10 (even) and 1 - 2^-11 -> 1 - 2^-10
      x/m = 2^-20       : a half subnormal (16 * 2^-24), exact
      x/m = 0.75*2^-24  : nearer 2^-24 than 0 -> 2^-24
      x/m = -0.5*2^-24  : halfway between -0 (even) and -2^-24 -> -0
      x/m = 0.1         : half 0x2E66 = 0.0999755859375
    """
    vals = np.array([2.0, 2 * (1 - 2.0 ** -12), 2 * (1 - 3 * 2.0 ** -12), 2 * 2.0 ** -20,
                     2 * 0.75 * 2.0 ** -24, -2 * 0.5 * 2.0 ** -24, 0.2, 0.0, 0.0, 0.0, 0.0, 0.0])
    want = np.array([2.0, 2.0, 2 * (1 - 2.0 ** -10), 2 * 2.0 ** -20, 2 * 2.0 ** -24, 0.0,
                     2 * 0.0999755859375, 0.0, 0.0, 0.0, 0.0, 0.0])
    site = (vals + 1j * vals[::-1]).reshape(1, 4, 3)
    got = solvers.round_storage(site, "f16").astype(np.complex128).reshape(-1)
    assert np.array_equal(got.real, want), got.real - want
    assert np.array_equal(got.imag, want[::-1]), got.imag - want[::-1]


def test_round_storage_f16_scale_and_bound():
    """On random fields of very different site magnitudes: each site's largest
    stored |real| equals its largest input |real| (after FP32 rounding) exactly,
    and every real is within (2^-12 + 2^-23) of that maximum of its input: the
    scaled values lie in [-1, 1], where half's largest rounding error is half
    an ulp of [1/2, 1), 2^-12; the FP32 product adds at most 2^-24 of m."""
    rng = np.random.default_rng(41)
    psi = rng.standard_normal((500, 4, 3)) + 1j * rng.standard_normal((500, 4, 3))
    psi *= 10.0 ** rng.uniform(-12, 6, size=(500, 1, 1))
    got = solvers.round_storage(psi, "f16").astype(np.complex128)
    c32 = psi.astype(np.complex64).astype(np.complex128)
    m_in = np.maximum(np.abs(c32.real), np.abs(c32.imag)).max(axis=(1, 2))
    m_out = np.maximum(np.abs(got.real), np.abs(got.imag)).max(axis=(1, 2))
    assert np.array_equal(m_in, m_out)
    err = np.maximum(np.abs(got.real - c32.real), np.abs(got.imag - c32.imag)).max(axis=(1, 2))
    assert np.all(err <= (2.0 ** -12 + 2.0 ** -23) * m_in)
    # the bound is reached to within a factor of two (rounding really happens)
    assert np.max(err / m_in) > 2.0 ** -13
    # a zero site stays zero
    assert np.all(solvers.round_storage(np.zeros((2, 4, 3), complex), "f16") == 0)
