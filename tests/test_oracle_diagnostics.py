"""Pins of the oracle's diagnostics (section IV interface length / domain size, eq. phiavg,
pressure of eq. pbin) against closed forms."""
import math

import numpy as np

from oracle import ref
from paper_1904_10070_amd import inputs


def grid_with(phi, n=None, r=1.0, R=2.5, A=0.5):
    nt, np_ = phi.shape
    g = ref.RefGrid(r, R, nt, np_, A, 1e-3, 0.1, 0.5, 1e-3)
    n0, ut, up = inputs.rest_moments(nt, np_)
    g.set_state(phi, n0 if n is None else n, ut, up)
    return g


def test_band_interface_length_is_two_circles():
    """phi = -1 on rows [q1, q2), +1 elsewhere: two interfaces at the half nodes q1 - 1/2 and
    q2 - 1/2, each a full circle of length 2 pi (R + r cos theta)."""
    nt, np_, r, R = 48, 30, 1.0, 2.5
    q1, q2 = 10, 29
    phi = np.ones((nt, np_))
    phi[q1:q2] = -1.0
    d = grid_with(phi, r=r, R=R).diagnostics()
    dth = 2 * math.pi / nt
    exact = 2 * math.pi * ((R + r * math.cos((q1 - 0.5) * dth)) + (R + r * math.cos((q2 - 0.5) * dth)))
    assert abs(d["L_I"] - exact) < 1e-12 * exact
    assert abs(d["A_total"] - 4 * math.pi ** 2 * r * R) < 1e-12


def test_checkerboard_interface_length():
    """every node differs from both neighbours: L_I = 2 pi (r N_phi + R N_theta)."""
    nt, np_, r, R = 24, 36, 0.8, 2.0
    q, s = np.meshgrid(np.arange(nt), np.arange(np_), indexing="ij")
    phi = np.where((q + s) % 2 == 0, 0.7, -0.7)
    d = grid_with(phi, r=r, R=R).diagnostics()
    assert abs(d["L_I"] - 2 * math.pi * (r * np_ + R * nt)) < 1e-10


def test_profiles_of_uniform_and_banded_fields():
    nt, np_, A = 16, 20, 0.5
    th = np.arange(nt) * 2 * np.pi / nt
    phi = np.repeat((0.9 * np.cos(th))[:, None], np_, axis=1)
    n = np.repeat((1 + 0.1 * np.sin(th))[:, None], np_, axis=1)
    d = grid_with(phi, n=n, A=A).diagnostics()
    ph = 0.9 * np.cos(th)
    assert np.allclose(d["phi_avg"], ph, rtol=0, atol=1e-14)
    assert np.allclose(d["p_avg"], 1 + 0.1 * np.sin(th) + A * (-0.5 * ph ** 2 + 0.75 * ph ** 4),
                       rtol=0, atol=1e-14)
    assert d["L_I"] > 0
