"""The learned preconditioner is trained on the GPU by the library's kernels,
survives a round trip through its weight checkpoint, and must beat the
method without it (FGCR with N = 1) on fresh sources."""
import numpy as np
import pytest

import paper_0710_2442_amd as wd
import synthetic as syn
from gpu_util import from_field, to_field
from paper_0710_2442_amd import learn
from oracle import solvers

pytestmark = pytest.mark.gpu


def test_training_reduces_loss_and_fgcr_iterations(tmp_path):
    dims, kappa = (8, 8, 8, 8), 0.124
    U = syn.gauge_field(dims, 0.3, 401)
    g = wd.Gauge(U, dims, -1, "f64")
    ck = tmp_path / "ptc.wdptc"
    W0, hist = learn.train(g, kappa, steps=200, batch=4, lr=3e-3, seed=7, act="bf16", log_every=20, checkpoint=ck)
    # the solves below use the network read back from its checkpoint
    W, meta = learn.load_weights(ck)
    assert np.array_equal(W, W0) and meta["dims"] == list(dims) and meta["steps"] == 200
    losses = [l for _, l in hist["losses"]]
    print("losses", losses, flush=True)
    assert losses[-1] < 0.7 * losses[0]
    # fresh source, not seen in training
    b = syn.gaussian_spinor(dims, 402)
    fb = to_field(g, b)
    res = {}
    for solver in (wd.WD_SOLVER_FGCR, wd.WD_SOLVER_DEFECT_FGCR):
        for name, net in (("identity", None), ("trained", wd.Ptc(g, W, "bf16"))):
            fx = wd.wd_new_field(dims, "f64")
            p = wd.wd_solve_params_default(solver=solver, fgcr_m=16 if solver == wd.WD_SOLVER_FGCR else 8,
                                           precond=net)
            rc, info = wd.wd_solve(g, fb, fx, kappa, 1e-10, p)
            assert rc == 0 and info["fallback_used"] == 0
            assert solvers.true_residual(U, b, from_field(g, fx), kappa) <= 1e-10
            res[(solver, name)] = info["iters"]
            if net is not None:
                net.close()
    print("fgcr iterations", res, flush=True)
    for solver in (wd.WD_SOLVER_FGCR, wd.WD_SOLVER_DEFECT_FGCR):
        assert res[(solver, "trained")] < 0.8 * res[(solver, "identity")]
    g.close()
