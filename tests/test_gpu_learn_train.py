"""What the trained network gains over the coarse step without it, with the fine solver as the
judge (spinodal coarsening, 512 x 1280 fine -> 128 x 320 coarse with a 4x time step).

The plain coarse grid keeps the fine interface width, which it cannot resolve: its interfaces
pin and its coarsening lengths fall behind the fine solution's (L_d about -9 %, the
structure-factor length L_S about -22 % four time units after the hand-over).  The tests train
a network from scratch on a reduced set of solver-made pairs and check the held-out one-step
loss and the judged L_S and L_d errors against the plain step's; and they check that the
committed weights (train_coarse.py) meet the stated bar of 2 % on a seed held out from their
training and selection.
"""
import numpy as np
import pytest

from paper_1904_10070_amd import inputs

pytestmark = pytest.mark.gpu

MASK = 13                       # phi and the velocity are corrected
LOSS_W = (1.0, 0.0, 0.25, 0.25)


def l_errors(rows, key="L"):
    """Largest relative error of the learned and of the plain coarse run for L_d (key "L") or
    the structure-factor length L_S (key "LS")."""
    e = [abs(r[key + "_learned"] - r[key + "_judge"]) / r[key + "_judge"] for r in rows]
    p = [abs(r[key + "_plain"] - r[key + "_judge"]) / r[key + "_judge"] for r in rows]
    return max(e), max(p)


@pytest.mark.timeout(400)
def test_training_from_scratch_gains_over_plain_coarse_step(torch_cuda):
    from paper_1904_10070_amd import learn as L
    pf = inputs.spinodal_workload(0.6)
    pc = L.coarse_params(pf)
    m, y = L.generate_shadow_pairs(pf, seeds=(1, 2), t_first=16.0, t_last=28.0, every=400,
                                   apply_mask=MASK)
    mv, yv = L.generate_shadow_pairs(pf, seeds=(4,), t_first=20.0, t_last=24.0, every=800,
                                     apply_mask=MASK)
    norm = L.normalisation(m, y)
    net = L.make_network(pc, norm, 16, seed=0, loss_weight=LOSS_W, apply_mask=MASK)
    before, zero = L.batch_loss(net, mv, yv)
    L.train(net, m, y, iters=2000, batch=16, lr=2e-3, seed=0, report_every=1000)
    after, _ = L.batch_loss(net, mv, yv)
    print(f"held-out one-step loss: plain step {zero:.3e}, untrained {before:.3e}, "
          f"trained {after:.3e}", flush=True)
    assert after < 0.05 * zero
    rows = L.evaluate(pf, net, seed=7, t_start=20.0, t_end=24.0, every_t=2.0)
    err, err_plain = l_errors(rows)
    errs, errs_plain = l_errors(rows, "LS")
    print(f"largest error over t in [20, 24]: L_d learned {err:.4f}, plain {err_plain:.4f}; "
          f"L_S learned {errs:.4f}, plain {errs_plain:.4f}", flush=True)
    assert all(r["nonfinite"] == 0 for r in rows)
    assert err < 0.5 * err_plain and errs < 0.5 * errs_plain
    assert rows[-1]["phi_l2_learned"] < rows[-1]["phi_l2_plain"]


@pytest.mark.timeout(300)
def test_committed_weights_meet_the_bar(torch_cuda):
    """Hand-over at t = 20 (seed 7, used neither for training nor for choosing the weights),
    judged to t = 30 (6250 coarse steps): the structure-factor length L_S and L_d within 2 % of
    those of the restricted fine solution, where the plain coarse step is off by more than 10 %
    (L_S: 30 %)."""
    from paper_1904_10070_amd import learn as L, train_coarse
    params, meta = train_coarse.load(0.6)
    assert 7 not in meta["recipe"]["train_seeds"] and meta["validation"]["seed"] != 7
    net = train_coarse.network_from(meta, params)
    pf = inputs.spinodal_workload(0.6)
    rows = L.evaluate(pf, net, seed=7, t_start=20.0, t_end=30.0, every_t=2.0)
    err, err_plain = l_errors(rows)
    errs, errs_plain = l_errors(rows, "LS")
    print(f"committed weights, seed 7, t in [20, 30]: largest error L_S learned {errs:.4f} "
          f"plain {errs_plain:.4f}, L_d learned {err:.4f} plain {err_plain:.4f}; phi L2 at "
          f"t=30 learned {rows[-1]['phi_l2_learned']:.3f} plain {rows[-1]['phi_l2_plain']:.3f}",
          flush=True)
    assert errs <= 0.02 and err <= 0.02 and err_plain > 0.10 and errs_plain > 0.10


@pytest.mark.timeout(300)
def test_runner_falls_back_to_the_fine_solver(torch_cuda):
    """Not accepted by the judge (a bar no network meets), or turning non-finite (weights
    blown up on purpose), the runner hands the run to the fine solver."""
    from paper_1904_10070_amd import TorusGrid, learn as L, train_coarse
    params, meta = train_coarse.load(0.6)
    pf = inputs.spinodal_workload(0.6)

    def fine_at(t):
        g = TorusGrid(pf, 32)
        g.set_state(inputs.spinodal_phi(pf, seed=9), *inputs.rest_moments(pf.n_theta, pf.n_phi))
        g.step(int(round(t / pf.dt)))
        return g

    net = train_coarse.network_from(meta, params)
    strict = L.LearnedCoarseRunner(pf, net, max_error=1e-9)
    strict.validate(seed=8, t_start=20.0, t_end=21.0, every_t=1.0, progress=None)
    assert not strict.accepted
    path, g = strict.run(fine_at(20.0), 0.4)
    assert path == "fine" and g.shape == (pf.n_theta, pf.n_phi)

    ok = L.LearnedCoarseRunner(pf, net, max_error=0.05)
    ok.validate(seed=8, t_start=20.0, t_end=21.0, every_t=1.0, progress=None)
    assert ok.accepted
    path, g = ok.run(fine_at(20.0), 0.4)
    assert path == "learned" and g.shape == (pf.n_theta // 4, pf.n_phi // 4)

    bad = train_coarse.network_from(meta, (params * 1e3).astype(np.float32))
    wild = L.LearnedCoarseRunner(pf, bad, max_error=1.0)
    wild.accepted = True          # skip the judge: the run itself must catch the blow-up
    path, g = wild.run(fine_at(20.0), 0.4)
    assert path == "fine" and g.invariants()[2] == 0
