"""Host side of the paper-experiment studies, on synthetic records whose answers are known: the
recorder's schedule (paper_1904_10070_amd/stripe.py), the oscillation fit and equilibrium
choice (tests/stripe_sweep.py), crossing counts and sides (tests/stripe_equilibrium.py), the
exponent fit (tests/coarsening.py) and the signed angles of the drop tracks."""
import math

import numpy as np

from paper_1904_10070_amd import inputs, stripe
from tests import coarsening, drop_drift, stripe_equilibrium, stripe_sweep


class FakeGrid:
    """Counts steps; its 'measurement' is the step count."""

    def __init__(self, dt):
        self.params = inputs.TorusParams(1.0, 2.0, 8, 8, 0.5, 1e-3, 1e-3, 0.1, dt)
        self.steps = 0

    def step(self, n):
        self.steps += n


def test_record_schedule():
    grids = [FakeGrid(0.01), FakeGrid(0.01)]
    calls = []

    def step(n):
        calls.append(n)
        for g in grids:
            g.step(n)

    t, recs = stripe.record(step, grids, 1.0, 0.25, lambda g: g.steps)
    assert np.allclose(t, [0.0, 0.25, 0.5, 0.75, 1.0])
    assert calls == [25, 25, 25, 25]
    assert recs == [[0, 25, 50, 75, 100]] * 2


def test_oscillation_analysis_recovers_a_synthetic_oscillation():
    """theta_c(t) = theta_eq + dtheta_0 cos(omega t) exp(-alpha t) with the closed-form
    equilibrium of the 0.28 pi stripe: the fits return omega and alpha."""
    p = stripe_sweep.torus(0.8, 320, 2.5e-3)
    th0, w0 = stripe_sweep.CASES["pi"]
    eq = stripe_sweep.st.predict(p.gamma, p.r, p.R, 1.0, p.tau, th0 * math.pi, w0 * math.pi)[0]
    t = np.arange(0.0, 601.0)
    omega, alpha = 0.083, 2.9e-3
    centre = eq["theta_c"] + (th0 * math.pi - eq["theta_c"]) * np.cos(omega * t) * np.exp(-alpha * t)
    r = stripe_sweep.analyse("pi", p, t, centre, np.full_like(t, eq["dtheta"]))
    assert abs(r["omega_fit"] / omega - 1) < 1e-4 and abs(r["alpha_fit"] / alpha - 1) < 1e-3
    assert abs(r["omega_free"] / omega - 1) < 1e-3 and abs(r["alpha_free"] / alpha - 1) < 1e-2
    assert r["finite"] and abs(r["theta_eq"] - math.pi) < 1e-12


def test_crossings_and_sides():
    c = math.pi + np.array([-0.3, -0.1, 0.2, 0.1, -0.05, -0.2, 0.0, 0.3])
    assert stripe_equilibrium.crossings(c) == 3      # the exact pi does not count twice
    assert stripe_equilibrium.side(math.pi + 0.005 * math.pi) == "pi"
    assert stripe_equilibrium.side(0.7 * math.pi) == "upper"
    assert stripe_equilibrium.side(1.3 * math.pi) == "lower"


def test_exponent_and_sampling():
    t = np.geomspace(1.0, 1000.0, 50)
    assert abs(coarsening.exponent(t, 0.1 * t ** (2 / 3), 40.0, 250.0) - 2 / 3) < 1e-12
    steps = coarsening.sample_steps(500.0, 5e-4)
    assert steps == sorted(set(steps)) and steps[0] == 2000 and steps[-1] == 1000000


def test_signed_angles():
    s = drop_drift.signed([0.1, 2 * math.pi - 0.1, math.pi, 3 * math.pi])
    assert np.allclose(s, [0.1, -0.1, -math.pi, -math.pi])
