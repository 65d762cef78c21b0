"""Pins of the oracle's WENO-5 advection variant (flag WENO5; the authors' earlier vielbein
scheme used WENO-5, the linear UW5 reading is its optimal-weight limit): reduction to UW5 when
the smoothness regulariser dominates, no overshoot at a discontinuity where UW5 overshoots,
fifth-order convergence of the advection operator on smooth data, exact conservation."""
import numpy as np

from oracle import ref
from paper_1904_10070_amd import inputs
from tests.test_oracle_operators import grid, smooth_populations


def test_weno_reduces_to_uw5_for_large_eps():
    rng = np.random.default_rng(0)
    for _ in range(50):
        h = rng.normal(size=5)
        assert abs(ref.weno5_face(h, eps=1e30) - ref.uw5_face(h)) <= 1e-13 * (1 + abs(ref.uw5_face(h)))
    # the linear face formula itself: (2, -13, 47, 27, -3) / 60
    assert abs(ref.uw5_face([1, 0, 0, 0, 0]) - 2 / 60) < 1e-16
    assert abs(ref.uw5_face([0, 0, 0, 1, 0]) - 27 / 60) < 1e-16


def test_weno_does_not_overshoot_a_step():
    up, down = [0, 0, 1, 1, 1], [1, 1, 0, 0, 0]
    assert abs(ref.uw5_face(up) - 71 / 60) < 1e-15 and abs(ref.uw5_face(down) + 11 / 60) < 1e-15
    assert abs(ref.weno5_face(up) - 1.0) < 1e-9 and abs(ref.weno5_face(down)) < 1e-9


def test_weno_advection_fifth_order_along_theta():
    r, R = 1.0, 2.5
    v, w, K, Kt = ref.velocity_set()
    errs = []
    for nt in (24, 48, 96, 192):
        g = grid(nt, 1, r=r, R=R, flags=ref.WENO5)
        th = np.arange(nt) * 2 * np.pi / nt
        J = R + r * np.cos(th)
        f, df = smooth_populations(nt, 1, "theta")
        adv = g.rhs_terms(f, np.zeros(g.shape))["adv"]
        exact = np.zeros_like(f)
        for k in range(16):
            exact[k] = -v[k // 4] / (r * J[:, None]) * (J[:, None] * df[k] - r * np.sin(th)[:, None] * f[k])
        errs.append(np.abs(adv - exact).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 4.6), rates


def test_weno_run_conserves_mass_and_phi():
    p = inputs.TorusParams(1.0, 2.5, 24, 40, 0.5, 2e-3, 0.05, 0.3, 2e-4, ref.WENO5)
    phi, n, ut, up = inputs.random_state(p, seed=21)
    g = ref.RefGrid(**p.as_dict())
    g.set_state(phi, n, ut, up)
    m0, s0, _ = g.invariants()
    g.step(60)
    m1, s1, bad = g.invariants()
    assert bad == 0 and abs(m1 - m0) < 1e-13 * m0 and abs(s1 - s0) < 1e-13 * m0
