"""GPU solves against the oracle.

Many x are correct: a solve passes when the oracle's own D_W applied to the
GPU solution gives |b - D x|/|b| <= 1e-10 (the FP64 true residual the library
reports must agree with it), and when the solution agrees with the oracle's
(or the exact free-field) solution within cond(D) * tol.
"""
import numpy as np
import pytest
import torch

import paper_0710_2442_amd as wd
import synthetic as syn
from gpu_util import from_field, rel_err, to_field
from oracle import free_field, solvers, wilson

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _solve(dims, kappa, eps, seed, **kw):
    U = syn.gauge_field(dims, eps, 1000 + seed)
    b = syn.gaussian_spinor(dims, 2000 + seed)
    g = wd.Gauge(U, dims, -1, "f64")
    fb = to_field(g, b)
    fx = wd.wd_new_field(dims, "f64")
    p = wd.wd_solve_params_default(**kw)
    rc, info = wd.wd_solve(g, fb, fx, kappa, TOL, p)
    x = from_field(g, fx)
    g.close()
    return U, b, x, rc, info


def test_fp64_cg_8x4_matches_oracle():
    """Plain FP64 Wilson-Dirac on 8^4, kappa = 0.12: CG on D^dag D to 1e-10."""
    dims, kappa = (8, 8, 8, 8), 0.12
    U, b, x, rc, info = _solve(dims, kappa, 0.3, 1, solver=wd.WD_SOLVER_CG)
    print("info", info, flush=True)
    assert rc == 0
    r_oracle = solvers.true_residual(U, b, x, kappa)
    assert r_oracle <= TOL
    assert abs(r_oracle - info["true_rel_resid"]) <= 1e-3 * TOL
    xo, it_o, _ = solvers.solve_eo_cgls(U, b, kappa, 1e-12)
    assert rel_err(x, xo) <= 1e-7  # cond(D) ~ 20 here
    # the GPU iteration count matches the oracle's eo-CGLS to within a few
    _, it_o10, _ = solvers.solve_eo_cgls(U, b, kappa, TOL)
    assert abs(info["iters"] - it_o10) <= 3, (info["iters"], it_o10)


@pytest.mark.parametrize("dims,use_graph", [((6, 4, 6, 10), 0), ((8, 8, 8, 8), 1)])
def test_full_lattice_cgls_matches_oracle(dims, use_graph):
    """CGLS on the full-lattice D_W (no even-odd reduction): the oracle's own
    D_W judges the residual, the solution agrees with the oracle's full CGLS
    (and with its even-odd solve), and the iteration count with the oracle's
    full CGLS to within a few (the same recurrence in another summation order)."""
    kappa = 0.12
    U, b, x, rc, info = _solve(dims, kappa, 0.3, 11, solver=wd.WD_SOLVER_CGLS_FULL, use_graph=use_graph,
                               check_every=4)
    print("info", info, flush=True)
    assert rc == 0
    r_oracle = solvers.true_residual(U, b, x, kappa)
    assert r_oracle <= TOL
    assert abs(r_oracle - info["true_rel_resid"]) <= 1e-3 * TOL
    xo, it_o, _ = solvers.solve_cgls_full(U, b, kappa, TOL)
    assert abs(info["iters"] - it_o) <= 3, (info["iters"], it_o)
    xe, _, _ = solvers.solve_eo_cgls(U, b, kappa, 1e-12)
    assert rel_err(x, xe) <= 1e-7
    # the full operator needs more iterations than the even-odd Schur system
    _, _, x2, rc2, info2 = _solve(dims, kappa, 0.3, 11, solver=wd.WD_SOLVER_CG)
    assert rc2 == 0 and info["iters"] > info2["iters"]


@pytest.mark.parametrize("solver", ["cgls_full", "fgcr"])
def test_full_lattice_solvers_on_the_one_launch_operator(solver):
    """32^3x8 is large enough that the full-lattice solvers apply D_W (and
    CGLS also D_W^dag, with its norm and convergence flag) through the
    one-launch marching kernel, whose work items then fill the device.  The
    oracle's D_W judges the residual; the solution agrees with the even-odd
    CG's."""
    dims, kappa = (32, 32, 32, 8), 0.12
    print(f"case: {solver} on the one-launch D_W, {dims}", flush=True)
    kw = dict(solver=wd.WD_SOLVER_CGLS_FULL, use_graph=1, check_every=4) if solver == "cgls_full" else \
        dict(solver=wd.WD_SOLVER_FGCR, fgcr_m=8)
    U, b, x, rc, info = _solve(dims, kappa, 0.3, 13, **kw)
    print("info", info, flush=True)
    assert rc == 0 and info["fallback_used"] == 0
    r = solvers.true_residual(U, b, x, kappa)
    assert r <= TOL and abs(r - info["true_rel_resid"]) <= 1e-3 * TOL
    _, _, x2, rc2, _ = _solve(dims, kappa, 0.3, 13, solver=wd.WD_SOLVER_CG)
    assert rc2 == 0 and rel_err(x, x2) <= 1e-7


@pytest.mark.parametrize("use_graph", [0, 1])
def test_fp64_cg_graph_and_eager_agree(use_graph):
    dims, kappa = (6, 4, 6, 10), 0.124
    U, b, x, rc, info = _solve(dims, kappa, 0.3, 2, solver=wd.WD_SOLVER_CG, use_graph=use_graph,
                               check_every=4)
    assert rc == 0 and solvers.true_residual(U, b, x, kappa) <= TOL


def test_graph_replays_bitwise_equal_to_eager():
    dims, kappa = (6, 4, 6, 10), 0.124
    outs = []
    for ug in (0, 1, 1):
        _, _, x, rc, info = _solve(dims, kappa, 0.3, 3, solver=wd.WD_SOLVER_CG, use_graph=ug, check_every=8)
        outs.append((x, info["iters"]))
    assert outs[0][1] == outs[1][1] == outs[2][1]
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[1][0], outs[2][0])


@pytest.mark.parametrize("prec,inner_tol", [("f32", 1e-4), ("f16", 1e-2), ("bf16", 1e-2)])
def test_defect_correction_reaches_fp64_residual(prec, inner_tol):
    dims, kappa = (8, 8, 8, 8), 0.124
    U, b, x, rc, info = _solve(dims, kappa, 0.3, 4, solver=wd.WD_SOLVER_DEFECT_CG, inner_prec=prec,
                               inner_tol=inner_tol)
    print(prec, info, flush=True)
    assert rc == 0
    r = solvers.true_residual(U, b, x, kappa)
    assert r <= TOL
    assert info["outer_iters"] >= 2
    xo, _, _ = solvers.solve_eo_cgls(U, b, kappa, 1e-12)
    assert rel_err(x, xo) <= 1e-6


def test_zero_source_and_kappa_zero():
    dims = (4, 4, 4, 4)
    U = syn.gauge_field(dims, 0.3, 5)
    g = wd.Gauge(U, dims, -1, "f64")
    fb = to_field(g, np.zeros(syn.lattice_shape(dims) + (4, 3), complex))
    fx = wd.wd_new_field(dims, "f64")
    rc, info = wd.wd_solve(g, fb, fx, 0.12, TOL)
    assert rc == 0 and np.all(from_field(g, fx) == 0)
    b = syn.gaussian_spinor(dims, 6)
    fb = to_field(g, b)
    rc, info = wd.wd_solve(g, fb, fx, 0.0, TOL)
    assert rc == 0 and rel_err(from_field(g, fx), b) < 1e-15
    g.close()


def test_nonfinite_source_is_rejected():
    dims = (4, 4, 4, 4)
    g = wd.Gauge(syn.gauge_field(dims, 0.3, 7), dims, -1, "f64")
    b = syn.gaussian_spinor(dims, 8)
    b[0, 0, 0, 0, 0, 0] = np.nan
    fb = to_field(g, b)
    fx = wd.wd_new_field(dims, "f64")
    with pytest.raises(wd.WdError) as e:
        wd.wd_solve(g, fb, fx, 0.12, TOL)
    assert e.value.status == -4
    g.close()


def test_iteration_cap_reports_not_converged():
    dims, kappa = (8, 8, 8, 8), 0.124
    U, b, x, rc, info = _solve(dims, kappa, 0.3, 9, solver=wd.WD_SOLVER_CG, max_iter=5)
    assert rc == 1 and info["iters"] <= 6
    assert info["true_rel_resid"] > TOL
    # x is still the reported iterate: its residual matches the oracle's
    assert abs(solvers.true_residual(U, b, x, kappa) - info["true_rel_resid"]) <= 1e-8


def test_free_field_solve_matches_fft_16x4():
    dims, kappa = (16, 16, 16, 16), 0.124
    U = syn.unit_gauge(dims)
    b = syn.gaussian_spinor(dims, 10)
    g = wd.Gauge(U, dims, -1, "f64")
    fb = to_field(g, b)
    fx = wd.wd_new_field(dims, "f64")
    for kw in (dict(solver=wd.WD_SOLVER_CG),
               dict(solver=wd.WD_SOLVER_DEFECT_CG, inner_prec="f16", inner_tol=1e-2)):
        rc, info = wd.wd_solve(g, fb, fx, kappa, TOL, wd.wd_solve_params_default(**kw))
        x = from_field(g, fx)
        xs = free_field.solve(b, kappa)
        assert rc == 0
        # cond(D) of the free operator on 16^4 at kappa = 0.124 is ~ 50
        assert rel_err(x, xs) <= 50 * TOL * 10, rel_err(x, xs)
    g.close()


def test_free_field_solves_at_full_size_32x32x32x64():
    """The solver workloads' lattice (32^3x64, kappa 0.124) with unit links,
    where the exact D^{-1} b is the oracle's FFT solution: plain FP64 CG,
    BF16-storage defect correction and the mixed even-odd FGCR (FP32 storage
    without a network; BF16 storage with a network, which then runs with
    FP16 products) must all land within cond(D) * tol of it.  Free-field
    cond(D) here is ~134 (lambda_min(D^dag D) = 2.2e-4)."""
    from paper_0710_2442_amd import learn

    dims, kappa = (32, 32, 32, 64), 0.124
    lo, hi = free_field.lambda_min_normal(dims, kappa)
    cond = np.sqrt(hi / lo)
    assert 130 < cond < 140
    U = syn.unit_gauge(dims)
    b = syn.gaussian_spinor(dims, 2003)
    g = wd.Gauge(U, dims, -1, "f64")
    del U
    fb = to_field(g, b)
    fx = wd.wd_new_field(dims, "f64")
    xs = free_field.solve(b, kappa)
    net = wd.Ptc(g, learn.init_weights(11, scale=0.05), "bf16")
    for kw in (dict(solver=wd.WD_SOLVER_CG),
               dict(solver=wd.WD_SOLVER_DEFECT_CG, inner_prec="bf16", inner_tol=1e-2),
               dict(solver=wd.WD_SOLVER_DEFECT_FGCR, fgcr_m=4, inner_tol=1e-2),
               dict(solver=wd.WD_SOLVER_DEFECT_FGCR, fgcr_m=4, inner_tol=1e-2, inner_prec="bf16", precond=net)):
        rc, info = wd.wd_solve(g, fb, fx, kappa, TOL, wd.wd_solve_params_default(**kw))
        assert rc == 0 and info["true_rel_resid"] <= TOL, (kw, info)
        err = rel_err(from_field(g, fx), xs)
        print(kw["solver"], info["iters"], info["true_rel_resid"], err, flush=True)
        assert err <= 2 * cond * TOL, (kw, err)
    net.close()
    g.close()


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_multi_rhs_point_sources(prec):
    """12 spin-colour point sources solved together (shared hop launches, own scalars)."""
    dims, kappa = (8, 8, 8, 8), 0.124
    U = syn.gauge_field(dims, 0.3, 1004)
    B = syn.point_sources(dims)  # (12, ...)
    g = wd.Gauge(U, dims, -1, "f64")
    fb = torch.cat([to_field(g, B[r]) for r in range(12)])
    fx = wd.wd_new_field(dims, "f64", 12)
    p = wd.wd_solve_params_default(solver=wd.WD_SOLVER_DEFECT_CG, inner_prec=prec, inner_tol=1e-3)
    rc, infos = wd.wd_solve_mrhs(g, fb, fx, 12, kappa, TOL, p)
    assert rc == 0
    nb = wd.wd_field_bytes(dims, "f64")
    for r in range(12):
        x = from_field(g, fx[r * nb:(r + 1) * nb])
        res = solvers.true_residual(U, B[r], x, kappa)
        assert res <= TOL, (r, res)
        assert abs(res - infos[r]["true_rel_resid"]) <= 1e-3 * TOL + 1e-14
    # a column of D^{-1}: compare one RHS with the single-RHS solve
    rc1, info1 = wd.wd_solve(g, fb[5 * nb:6 * nb], fx[:nb], kappa, TOL, p)
    x1 = from_field(g, fx[:nb])
    xo, _, _ = solvers.solve_eo_cgls(U, B[5], kappa, 1e-12)
    assert rel_err(x1, xo) <= 1e-6
    g.close()


def test_multi_rhs_solve_beyond_one_chunk():
    """24 Gaussian sources in one multi-RHS solve (BF16 storage; more RHS than
    one chunk of the multi-RHS hop, the count the training uses): every
    system reaches the tolerance by the oracle's own D_W."""
    dims, kappa, n = (8, 4, 6, 8), 0.124, 24
    U = syn.gauge_field(dims, 0.3, 31)
    bs = syn.gaussian_spinor(dims, 32, nrhs=n)
    g = wd.Gauge(U, dims, -1, "f64")
    fb = torch.cat([to_field(g, bs[r]) for r in range(n)])
    fx = wd.wd_new_field(dims, "f64", n)
    p = wd.wd_solve_params_default(solver=wd.WD_SOLVER_DEFECT_CG, inner_prec="bf16", inner_tol=1e-2)
    rc, infos = wd.wd_solve_mrhs(g, fb, fx, n, kappa, TOL, p)
    assert rc == 0
    nb = wd.wd_field_bytes(dims, "f64")
    for r in range(n):
        res = solvers.true_residual(U, bs[r], from_field(g, fx[r * nb:(r + 1) * nb]), kappa)
        assert res <= TOL, (r, res)
    g.close()


def test_multi_rhs_mixed_convergence_masks():
    """Systems that converge early stop consuming work; others continue to tolerance."""
    dims, kappa = (6, 4, 6, 10), 0.124
    U = syn.gauge_field(dims, 0.3, 11)
    bs = syn.gaussian_spinor(dims, 12, nrhs=3)
    bs[1] *= 0.0  # a zero right-hand side converges at once
    g = wd.Gauge(U, dims, -1, "f64")
    fb = torch.cat([to_field(g, bs[r]) for r in range(3)])
    fx = wd.wd_new_field(dims, "f64", 3)
    p = wd.wd_solve_params_default(solver=wd.WD_SOLVER_DEFECT_CG, inner_prec="f32", inner_tol=1e-4)
    rc, infos = wd.wd_solve_mrhs(g, fb, fx, 3, kappa, TOL, p)
    assert rc == 0
    nb = wd.wd_field_bytes(dims, "f64")
    assert np.all(from_field(g, fx[nb:2 * nb]) == 0)
    for r in (0, 2):
        assert solvers.true_residual(U, bs[r], from_field(g, fx[r * nb:(r + 1) * nb]), kappa) <= TOL
    g.close()
