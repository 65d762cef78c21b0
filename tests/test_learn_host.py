"""Host-side pieces of the learned coarse step that need no GPU: the committed weights and
the coarse-grid parameters."""
import numpy as np

from oracle import cnn_ref as C
from paper_1904_10070_amd import inputs, learn as L


def test_stored_weights_metadata():
    """The committed weights of the learned coarse step: right size, finite, and a recipe whose
    training and validation seeds leave the evaluation seed 7 out."""
    from paper_1904_10070_amd import train_coarse
    params, meta = train_coarse.load(0.6)
    assert params.dtype == np.float32 and params.size == C.param_count()
    assert np.all(np.isfinite(params))
    assert meta["coarse"]["n_theta"] * 4 == meta["fine"]["n_theta"] == 512
    assert meta["coarse"]["n_phi"] * 4 == meta["fine"]["n_phi"] == 1280
    assert abs(meta["coarse"]["dt"] - 4 * meta["fine"]["dt"]) < 1e-15
    assert 7 not in meta["recipe"]["train_seeds"] and meta["validation"]["seed"] != 7
    assert all(s > 0 for s in meta["out_scale"]) and all(s > 0 for s in meta["in_scale"])


def test_coarse_params_keep_physics_and_scale_grid_and_step():
    pf = inputs.spinodal_workload(0.6)
    pc = L.coarse_params(pf)
    assert (pc.n_theta, pc.n_phi) == (128, 320) and abs(pc.dt - 4 * pf.dt) < 1e-15
    assert (pc.kappa, pc.A, pc.M, pc.tau, pc.r, pc.R) == (pf.kappa, pf.A, pf.M, pf.tau, pf.r, pf.R)
    assert L.coarse_params(pf, kappa=2 * pf.kappa).kappa == 2 * pf.kappa
