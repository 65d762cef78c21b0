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


# -- structure-factor length (oracle/structure.py) ------------------------------------------

def brute_structure(phi, r, R):
    """The definition written out: a double loop over modes and nodes."""
    H, W = phi.shape
    d = phi - phi.mean()
    s0 = s1 = 0.0
    for m in range(H):
        mm = m if m <= H // 2 - (1 if H % 2 == 0 else 0) else m - H
        if H % 2 == 0 and m == H // 2:
            mm = -H // 2
        for mp in range(W):
            mmp = mp if mp < (W + 1) // 2 else mp - W
            acc = 0j
            for q in range(H):
                for s in range(W):
                    acc += d[q, s] * np.exp(-2j * np.pi * (m * q / H + mp * s / W))
            S = abs(acc) ** 2
            s0 += S
            s1 += np.hypot(mm / r, mmp / R) * S
    return 2 * np.pi * s0 / s1


def test_structure_length_definition_and_closed_forms():
    from oracle import structure as S
    rng = np.random.default_rng(3)
    phi = rng.uniform(-1, 1, (6, 10))
    assert abs(S.structure_length(phi, 1.0, 2.5)[0] - brute_structure(phi, 1.0, 2.5)) < 1e-12
    H, W, r, R = 32, 48, 1.0, 2.5
    th = 2 * np.pi * np.arange(H) / H
    ph = 2 * np.pi * np.arange(W) / W
    # a single mode: all power at |k| = 3 / r, or 2 / R, or sqrt((3/r)^2 + (2/R)^2)
    assert abs(S.structure_length(np.cos(3 * th)[:, None] + 0 * ph, r, R)[0] - 2 * np.pi * r / 3) < 1e-12
    assert abs(S.structure_length(0 * th[:, None] + np.cos(2 * ph), r, R)[0] - np.pi * R) < 1e-12
    both = np.cos(3 * th)[:, None] * np.cos(2 * ph)[None, :]
    assert abs(S.structure_length(both, r, R)[0] - 2 * np.pi / np.hypot(3 / r, 2 / R)) < 1e-12
    # Parseval: sum S = N sum (phi - <phi>)^2
    d = phi - phi.mean()
    assert abs(S.structure_length(phi, 1.0, 2.5)[1] - phi.size * (d * d).sum()) < 1e-10
