"""Drift of stripes and drops at the paper's parameters on the GPU, FP64 and FP32 (section III C
and D of the paper).

Stripes (r = 0.8, R = 2, kappa = 5e-4, A = 0.5, dt = 5e-4), started pi/20 from equilibrium,
oscillate about it as eq. stripe_hydro_sol says.  The fitted frequency is compared with eqs.
stripe_hydro_omega0_pi / _npi.  The damping rate is alpha_nu of eq. stripe_alphanu plus a part
that does not depend on nu: raising nu at a fixed mobility M raises the rate by exactly the
change of alpha_nu, while the rest falls with the grid spacing (about h^2 / M: it is the
friction of the interface, two cells wide at N_theta = 320, on the grid) -- the paper neglects
everything but alpha_nu.  Drops (r = 0.8, R = 2, 256 x 640, kappa = 5e-4, A = 0.5,
tau = M = 2.5e-3, eq. drop_init with the printed (theta_0, R_0)): they move to the outer
equator theta = 0, overshoot it and oscillate about it with a decaying amplitude.
"""
import math

import numpy as np
import pytest

from tests import drop_drift, stripe_sweep

pytestmark = pytest.mark.gpu


def oscillation_configs():
    """Both equilibria, nu = 2.5e-3 and 7.5e-3 at M = 2.5e-3 on N_theta = 320, and the first
    again on N_theta = 480."""
    cfgs = [(case, stripe_sweep.torus(0.8, 320, nu, M=2.5e-3))
            for case in ("pi", "3pi/4") for nu in (2.5e-3, 7.5e-3)]
    return cfgs + [("pi", stripe_sweep.torus(0.8, 480, 2.5e-3, M=2.5e-3))]


@pytest.mark.timeout(400)
def test_stripe_oscillation_against_closed_forms(torch_cuda):
    cfgs = oscillation_configs()
    res = {prec: stripe_sweep.run(cfgs, prec, 600.0) for prec in (64, 32)}
    for prec in (64, 32):
        print(f"FP{prec}\n" + stripe_sweep.table(res[prec]), flush=True)
    for x64, x32 in zip(res[64], res[32]):
        assert x64["finite"] and x32["finite"]
        assert abs(x64["omega_fit"] / x64["omega0"] - 1) <= 0.05, x64
        assert x64["alpha_fit"] > x64["alpha_nu"], x64
        assert abs(x64["theta_end"] - x64["theta_eq"]) <= 0.01 * math.pi, x64
        assert abs(x32["omega_fit"] / x64["omega_fit"] - 1) <= 0.01, (x32, x64)
        assert abs(x32["alpha_fit"] / x64["alpha_fit"] - 1) <= 0.1, (x32, x64)
        assert x64["mass_drift"] < 1e-9 and x32["mass_drift"] < 1e-5
    r = res[64]
    for lo, hi in ((r[0], r[1]), (r[2], r[3])):     # nu = 2.5e-3 and 7.5e-3, same M
        slope = (hi["alpha_fit"] - lo["alpha_fit"]) / (hi["alpha_nu"] - lo["alpha_nu"])
        print(f"{lo['case']}: d alpha / d alpha_nu = {slope:.3f}", flush=True)
        assert abs(slope - 1) <= 0.1
    excess = [x["alpha_fit"] - x["alpha_nu"] for x in (r[0], r[4])]   # N_theta 320, 480
    print(f"damping beyond alpha_nu: N_theta 320 {excess[0]:.2e}, 480 {excess[1]:.2e}", flush=True)
    assert excess[1] < 0.5 * excess[0]


@pytest.mark.timeout(400)
def test_drops_drift_to_the_outer_equator(torch_cuda):
    tracks = {}
    for prec in (64, 32):
        t, tracks[prec], drift = drop_drift.run(prec, 300.0)
        print(f"FP{prec}: theta_c / pi every 25 time units: " +
              "; ".join(" ".join(f"{x / math.pi:+.3f}" for x in s[::25]) for s in tracks[prec]) +
              f"; largest mass drift {max(drift):.1e}", flush=True)
        assert max(drift) < (1e-9 if prec == 64 else 1e-5)
    for (th0, _), s64, s32 in zip(drop_drift.DROPS, tracks[64], tracks[32]):
        assert abs(s64[0] - th0 * math.pi) < 0.05 * math.pi
        first = int(np.argmax(s64 <= 0.0))            # first record at or past the outer equator
        assert s64[first] <= 0.0 and t[first] < 150.0, (th0, t[first])
        assert np.all(np.diff(s64[:first + 1]) < 0.0), th0    # straight there, over the top
        late = t >= 200.0
        swing = np.abs(s64[first:][~late[first:]]).max()
        assert s64[first:].min() < -0.05 * math.pi, th0        # overshoot
        assert np.abs(s64[late]).max() < 0.6 * swing, th0      # decaying oscillation
        assert np.abs(s32 - s64).max() < 0.02 * math.pi, th0


@pytest.mark.timeout(400)
def test_fourth_order_cahn_hilliard_damps_stripes_closer_to_alpha_nu(torch_cuda):
    """The damping beyond alpha_nu at N_theta = 320 (the interface friction of the
    second-order Cahn-Hilliard discretisation, two cells per xi_0) is cut by the fourth-order
    variant TLB_CH4: the pi case at nu = M = 2.5e-3, FP64, t <= 600.  Measured 2.3e-3 against
    5.0e-4 (alpha / alpha_nu 4.1 against 1.7); bar: below 0.4 of the second-order excess, with
    the frequency within 5 % of omega_0."""
    cfgs = [("pi", stripe_sweep.torus(0.8, 320, 2.5e-3)),
            ("pi", stripe_sweep.torus(0.8, 320, 2.5e-3, flags=stripe_sweep.CH4))]
    ch2, ch4 = stripe_sweep.run(cfgs, 64, 600.0)
    print(stripe_sweep.table([ch2, ch4]), flush=True)
    ex2, ex4 = (x["alpha_fit"] - x["alpha_nu"] for x in (ch2, ch4))
    assert ch4["finite"] and abs(ch4["omega_fit"] / ch4["omega0"] - 1) <= 0.05
    assert abs(ch4["theta_end"] - ch4["theta_eq"]) <= 0.01 * math.pi
    assert ch4["mass_drift"] < 1e-9
    assert 0 < ex4 < 0.4 * ex2, (ex2, ex4)
