"""Closed-form predictions for stripes on a torus, and the field measurements compared to them.

TEST INFRASTRUCTURE ONLY.  The formulas are those printed in section III of the paper:
  stripe area (eq. stripe_area), interface length (eq. stripe_ltot), the equilibrium
  condition (eq. minimaring), the critical area (eq. stripe_dA_crit), the two equilibria above
  it (eq. stripe_thceq), the Laplace pressure (eqs. stripe_laplace_gen, stripe_laplace_eq),
  the viscous damping rate (eq. stripe_alphanu) and the oscillation frequencies
  (eqs. stripe_hydro_omega0_pi, stripe_hydro_omega0_npi).
The stripe is the minority phase (phi < 0 in the paper's convention), of angular width
dtheta and centre theta_c.
"""
import math

import numpy as np
from scipy.optimize import brentq


def stripe_area(r, R, theta_c, dtheta):
    a = r / R
    return 2 * math.pi * r * R * (dtheta + 2 * a * math.sin(dtheta / 2) * math.cos(theta_c))


def interface_length(r, R, theta_c, dtheta):
    a = r / R
    return 4 * math.pi * R * (1 + a * math.cos(theta_c) * math.cos(dtheta / 2))


def critical_area(r, R):
    a = r / R
    return 4 * math.pi * r * R * (math.acos(a) - a * math.sqrt(1 - a * a))


def equilibria(r, R, area):
    """Equilibrium (theta_c, dtheta) pairs for a stripe of the given area.

    Below the critical area: one equilibrium at theta_c = pi.  Above it: cos(dtheta/2) =
    -a cos(theta_c), and the area becomes 2 pi r R (dtheta - sin dtheta); two mirror
    equilibria pi -/+ arccos(cos(dtheta/2)/a).
    """
    a = r / R
    if area < critical_area(r, R):
        g = lambda d: 2 * math.pi * r * R * (d - 2 * a * math.sin(d / 2)) - area
        d = brentq(g, 1e-12, 2 * math.pi)
        return [(math.pi, d)]
    g = lambda d: 2 * math.pi * r * R * (d - math.sin(d)) - area
    d = brentq(g, 1e-12, 2 * math.pi)
    off = math.acos(max(-1.0, min(1.0, math.cos(d / 2) / a)))
    return [(math.pi - off, d), (math.pi + off, d)]


def laplace_pressure(gamma, r, R, theta_c, dtheta):
    """Pressure inside minus outside the stripe (eq. stripe_laplace_gen)."""
    a = r / R
    return (-gamma / R * math.cos(theta_c) * math.sin(dtheta / 2) /
            (1 + a * math.cos(theta_c) * math.cos(dtheta / 2)))


def alpha_nu(nu, r, R):
    return nu / (R * R - r * r)


def omega0(gamma, r, R, n, theta_c_eq, dtheta_eq, m=1.0):
    """Oscillation frequency about an equilibrium (subcritical: theta_c = pi)."""
    a = r / R
    if abs(theta_c_eq - math.pi) < 1e-9:
        c = math.cos(dtheta_eq / 2)
        w2 = gamma * math.sqrt(1 - a * a) / (math.pi * r * r * R * n * m) * (c - a) / (1 - a * c) ** 3
    else:
        w2 = (2 * gamma / (math.pi * r * R * R * n * m * (1 - a * a) ** 1.5) *
              (math.sin(theta_c_eq) / math.sin(dtheta_eq / 2)) ** 2)
    return math.sqrt(w2)


def predict(gamma, r, R, n, nu, theta0, dtheta0):
    """All equilibria of a stripe started at (theta0, dtheta0), with their dp and omega0."""
    area = stripe_area(r, R, theta0, dtheta0)
    out = []
    for tc, d in equilibria(r, R, area):
        out.append(dict(theta_c=tc, dtheta=d, dp=laplace_pressure(gamma, r, R, tc, d),
                        omega0=omega0(gamma, r, R, n, tc, d), alpha=alpha_nu(nu, r, R),
                        area=area, area_ratio=area / critical_area(r, R)))
    return out


# -- measurements on a field ------------------------------------------------------------------

def stripe_centre(phi, minority_sign=-1.0):
    """Centre and width of the stripe from the azimuthal average <phi>(theta) (eq. phiavg).

    The two zero crossings of <phi> are located by linear interpolation; the stripe is the arc
    on which minority_sign * <phi> > 0, and its centre is the arc's circular midpoint.
    Returns (theta_c, dtheta), or None if there are not exactly two crossings.
    """
    prof = minority_sign * np.asarray(phi).mean(axis=1)
    nt = prof.size
    dth = 2 * math.pi / nt
    cross = []  # (theta of crossing, entering the stripe?)
    for q in range(nt):
        a, b = prof[q], prof[(q + 1) % nt]
        if (a > 0) != (b > 0):
            t = (q + a / (a - b)) * dth
            cross.append((t % (2 * math.pi), b > 0))
    if len(cross) != 2:
        return None
    t_in = [t for t, entering in cross if entering][0]
    t_out = [t for t, entering in cross if not entering][0]
    width = (t_out - t_in) % (2 * math.pi)
    return (t_in + width / 2) % (2 * math.pi), width


def total_pressure(n, phi, A):
    """p = n k_B T + p_binary with p_binary = A(-phi^2/2 + 3 phi^4/4) (eq. pbin)."""
    return n + A * (-0.5 * phi ** 2 + 0.75 * phi ** 4)


def measured_laplace_pressure(n, phi, A, theta_c):
    """p at the node nearest theta_c minus p at the node nearest theta_c + pi, phi-averaged."""
    nt = phi.shape[0]
    p = total_pressure(n, phi, A).mean(axis=1)
    qi = int(round(theta_c / (2 * math.pi) * nt)) % nt
    qo = (qi + nt // 2) % nt
    return float(p[qi] - p[qo])


def fit_damped_oscillation_window(t, dtheta, omega_guess, alpha_guess, t_min):
    """Least squares of A cos(omega t + s) exp(-alpha t) + c over the samples with t >= t_min.

    Amplitude, phase and offset are free; the early part of the record, where the initial
    tanh profile relaxes to the torus equilibrium profile, is left out.  Returns
    (omega, alpha).
    """
    from scipy.optimize import least_squares
    t = np.asarray(t, float)
    y = np.asarray(dtheta, float)
    m = t >= t_min
    tt, yy = t[m], y[m]

    def res(x):
        A, w, ph, al, c = x
        return A * np.cos(w * tt + ph) * np.exp(-al * tt) + c - yy

    best = None
    for ph0 in np.linspace(0, 2 * np.pi, 8, endpoint=False):
        s = least_squares(res, [np.abs(yy).max(), omega_guess, ph0, alpha_guess, 0.0])
        if best is None or s.cost < best.cost:
            best = s
    return float(best.x[1]), float(best.x[3])


def fit_damped_oscillation(t, dtheta, dtheta0):
    """Least squares of dtheta0 cos(omega t) exp(-alpha t) (eq. stripe_hydro_sol, phase 0)."""
    from scipy.optimize import least_squares
    t = np.asarray(t, float)
    y = np.asarray(dtheta, float)

    def res(x):
        w, al = x
        return dtheta0 * np.cos(w * t) * np.exp(-al * t) - y

    # initial guess for omega from the first zero crossing
    sgn = np.sign(y)
    idx = np.nonzero(sgn[1:] != sgn[:-1])[0]
    w0 = math.pi / 2 / t[idx[0] + 1] if idx.size else 2 * math.pi / (t[-1] + 1e-30)
    sol = least_squares(res, x0=[w0, 1e-3], bounds=([0, -1], [np.inf, np.inf]))
    return float(sol.x[0]), float(sol.x[1])


def minority_centroid_theta(phi, J, minority_sign=-1.0):
    """theta of the area-weighted circular centroid of the minority phase (a drop's centre).

    Weight (1 - minority_sign * ... ) / 2 clipped to [0, 1], i.e. the local fraction of the
    minority phase, times the area element J (the common factor r dtheta dphi drops out)."""
    phi = np.asarray(phi)
    nt = phi.shape[0]
    th = np.arange(nt) * 2 * math.pi / nt
    wgt = np.clip((1 + minority_sign * phi) / 2, 0, 1) * np.asarray(J)[:, None]
    z = (wgt * np.exp(1j * th)[:, None]).sum()
    return math.atan2(z.imag, z.real) % (2 * math.pi)
