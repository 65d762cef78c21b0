"""Pins of the oracle's fourth-order Cahn-Hilliard variant (flag CH4): each operator against
closed forms of the torus geometry (appendix A: g_theta-theta = r^2, g_phi-phi = J^2,
J = R + r cos theta) with the convergence order measured, exact discrete symbols, and the
conservation of the area-weighted sum (the operators are differences of face quantities).

  Delta_S h = 1/(r^2 J) d_theta (J d_theta h) + 1/J^2 d_phi^2 h (eq. mu, eq. CH)
  div V = 1/(r J) d_theta (J V^theta) + 1/J d_phi V^phi (eq. CH, advection of phi)
"""
import math

import numpy as np

from oracle import ref
from paper_1904_10070_amd import inputs

R0, r0 = 2.5, 1.0


def grid(nt, np_, flags=ref.CH4, A=0.0, kappa=1.0, M=0.0):
    return ref.RefGrid(r0, R0, nt, np_, A, kappa, M, 0.5, 1e-4, flags)


def angles(nt, np_):
    th = np.arange(nt) * 2 * math.pi / nt
    ph = np.arange(np_) * 2 * math.pi / np_
    return np.meshgrid(th, ph, indexing="ij")


def laplacian(g, h, nt, np_):
    """Delta_S h from the oracle: with A = 0 and kappa = 1, mu = -Delta_S h."""
    g.set_state(h, *inputs.rest_moments(nt, np_))
    f, _ = g.get_state()
    return g.rhs_terms(f, h)["lap"]


def test_laplacian_of_cos_theta_converges_at_fourth_order():
    """Delta_S cos theta = -(R cos theta + r cos 2 theta) / (r^2 J): the error falls 16-fold
    per halving of the spacing (second order: 4-fold, checked alongside)."""
    errs4, errs2 = [], []
    for nt in (32, 64, 128):
        T, _ = angles(nt, 1)
        h = np.cos(T)
        exact = -(R0 * np.cos(T) + r0 * np.cos(2 * T)) / (r0 ** 2 * (R0 + r0 * np.cos(T)))
        errs4.append(np.abs(laplacian(grid(nt, 1), h, nt, 1) - exact).max())
        errs2.append(np.abs(laplacian(grid(nt, 1, flags=0), h, nt, 1) - exact).max())
    r4 = np.array(errs4[:-1]) / np.array(errs4[1:])
    r2 = np.array(errs2[:-1]) / np.array(errs2[1:])
    assert np.all((r4 > 14) & (r4 < 18)), (errs4, r4)
    assert np.all((r2 > 3.5) & (r2 < 4.5)), (errs2, r2)
    assert errs4[-1] < 1e-6


def test_laplacian_along_phi_has_the_exact_fourth_order_symbol():
    """cos(m phi) is an eigenfunction of the discrete operator with eigenvalue
    (-2 cos 2 m d + 32 cos m d - 30) / (12 d^2 J^2), d = dphi (five-point fourth order)."""
    nt, np_ = 6, 40
    T, P = angles(nt, np_)
    d = 2 * math.pi / np_
    J = R0 + r0 * np.cos(T)
    for m in (1, 3, 7, 20):
        h = np.cos(m * P)
        lam = (-2 * math.cos(2 * m * d) + 32 * math.cos(m * d) - 30) / (12 * d * d)
        got = laplacian(grid(nt, np_), h, nt, np_)
        assert np.abs(got - lam * h / J ** 2).max() <= 1e-12 * abs(lam) / (R0 - r0) ** 2, m


def test_laplacian_conserves_the_area_weighted_sum():
    """sum_q,s J_q (Delta_S h)_q,s = 0 to round-off for any h (the operator is a difference of
    face fluxes), on a ragged grid with wrap-around stencils."""
    nt, np_ = 23, 37
    rng = np.random.default_rng(3)
    h = rng.uniform(-1, 1, (nt, np_))
    lap = laplacian(grid(nt, np_), h, nt, np_)
    T, _ = angles(nt, np_)
    J = R0 + r0 * np.cos(T)
    assert abs((J * lap).sum()) <= 1e-11 * (J * np.abs(lap)).sum()


def div_case(nt, np_):
    """phi = cos theta + sin 2 phi, u^theta = 0.01 cos phi, u^phi = 0.02 sin theta (n = 1) and
    the closed form of -div(u phi)."""
    T, P = angles(nt, np_)
    J = R0 + r0 * np.cos(T)
    phi = np.cos(T) + np.sin(2 * P)
    a, b = 0.01, 0.02
    ut, up = a * np.cos(P), b * np.sin(T)
    d_th = a * np.cos(P) * (-r0 * np.sin(T) * phi + J * (-np.sin(T)))  # d_theta(J u^theta phi)
    d_ph = b * np.sin(T) * 2 * np.cos(2 * P)                          # d_phi(u^phi phi)
    exact = -(d_th / (r0 * J) + d_ph / J)
    return phi, np.ones_like(phi), ut, up, exact


def test_advection_divergence_converges_at_fourth_order():
    """With M = 0, L_phi = -div(u phi); the error falls 16-fold per halving in both angles."""
    errs = []
    for nt in (32, 64, 128):
        np_ = 2 * nt
        phi, n, ut, up, exact = div_case(nt, np_)
        g = grid(nt, np_, kappa=0.0)
        g.set_state(phi, n, ut, up)
        f, _ = g.get_state()
        errs.append(np.abs(g.rhs_terms(f, phi)["Lphi"] - exact).max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all((ratios > 14) & (ratios < 18)), (errs, ratios)


def test_force_gradient_converges_at_fourth_order():
    """F = -phi grad mu / n with mu = -Delta_S phi (A = 0, kappa = 1) for phi = cos theta:
    grad^theta-hat mu = (1/r) d_theta mu against the derivative of the closed form of mu."""
    errs = []
    for nt in (32, 64, 128):
        T, _ = angles(nt, 1)
        phi = np.cos(T)
        J = R0 + r0 * np.cos(T)
        # mu = (R cos + r cos 2) / (r^2 J); d_theta mu by the quotient rule
        num = R0 * np.cos(T) + r0 * np.cos(2 * T)
        dnum = -R0 * np.sin(T) - 2 * r0 * np.sin(2 * T)
        dmu = (dnum * J - num * (-r0 * np.sin(T))) / (r0 ** 2 * J ** 2)
        exact = -phi * dmu / r0
        g = grid(nt, 1)
        g.set_state(phi, *inputs.rest_moments(nt, 1))
        f, _ = g.get_state()
        errs.append(np.abs(g.rhs_terms(f, phi)["Fth"] - exact).max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all((ratios > 14) & (ratios < 18)), (errs, ratios)


def test_fourth_order_step_conserves_mass_and_phi():
    """A random state stepped 300 times with the fourth-order Cahn-Hilliard operators: mass and
    the area-weighted sum of phi stay at their initial values to 1e-13 (relative to the mass)."""
    p = inputs.TorusParams(1.0, 2.5, 24, 60, 0.5, 2e-3, 0.05, 0.3, 2e-4, ref.CH4)
    g = ref.RefGrid(**p.as_dict())
    g.set_state(*inputs.random_state(p, seed=8))
    m0, s0, _ = g.invariants()
    g.step(300)
    m1, s1, bad = g.invariants()
    assert bad == 0
    assert abs(m1 - m0) <= 1e-13 * m0 and abs(s1 - s0) <= 1e-13 * m0, (m1 - m0, s1 - s0)


def test_planar_profile_chemical_potential_vanishes_at_fourth_order():
    """The tanh band of width xi_0 = sqrt(kappa / A) is stationary in the continuum; its
    discrete mu falls 16-fold per halving of the spacing (4-fold with the second-order
    operator), flat limit."""
    mus = []
    for nt in (128, 256, 512):
        p = inputs.TorusParams(1.0, 2.0, nt, 1, 0.5, 5e-3, 0.01, 0.1, 5e-4, ref.FLAT | ref.CH4)
        phi = inputs.stripe_phi(p, math.pi, math.pi, offset=False)
        g = ref.RefGrid(**p.as_dict())
        g.set_state(phi, *inputs.rest_moments(nt, 1))
        mus.append(np.abs(g.moments()["mu"]).max())
    ratios = np.array(mus[:-1]) / np.array(mus[1:])
    assert np.all((ratios > 13) & (ratios < 19)), (mus, ratios)
