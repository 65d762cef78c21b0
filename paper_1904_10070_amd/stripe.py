"""Stripe measurements from the GPU diagnostics (section III of the paper): the band's centre
theta_c and angular width from the azimuthal average <phi>(theta) (eq. phiavg), and the
Laplace pressure as the difference of the azimuthally averaged pressure
p = n + A(-phi^2/2 + 3 phi^4/4) (eq. pbin) across the torus, at the node nearest theta_c and
the node opposite it (theta_c + pi).  The profiles come from tlb_diagnostics; only the search
for the two sign changes runs here, on n_theta host values.
"""
import math

import numpy as np


def centre_and_width(phi_avg, band_sign=1.0):
    """(theta_c, width) of the arc on which band_sign * <phi> > 0, from the two sign changes
    of <phi>(theta) located by linear interpolation between nodes; None unless there are
    exactly two."""
    prof = band_sign * np.asarray(phi_avg, dtype=np.float64)
    nt = prof.size
    h = 2.0 * math.pi / nt
    start = end = None
    count = 0
    for q in range(nt):
        a, b = prof[q], prof[(q + 1) % nt]
        if (a > 0.0) == (b > 0.0):
            continue
        count += 1
        theta = ((q + a / (a - b)) * h) % (2.0 * math.pi)
        if b > 0.0:
            start = theta       # entering the band
        else:
            end = theta         # leaving it
    if count != 2:
        return None
    width = (end - start) % (2.0 * math.pi)
    return (start + 0.5 * width) % (2.0 * math.pi), width


def laplace_pressure(p_avg, theta_c):
    """<p> at the node nearest theta_c minus <p> at the node opposite it."""
    p = np.asarray(p_avg, dtype=np.float64)
    nt = p.size
    qi = int(round(theta_c / (2.0 * math.pi) * nt)) % nt
    return float(p[qi] - p[(qi + nt // 2) % nt])


def track(grid, t_end, every_t, band_sign=1.0):
    """Advance `grid` (a TorusGrid) to t_end, recording (t, theta_c, width, dp) every every_t
    of simulated time.  Returns four numpy arrays (NaN where the band is not found)."""
    dt = grid.params.dt
    n_every = int(round(every_t / dt))
    rows = []
    steps = 0
    while steps * dt < t_end - 0.5 * dt:
        grid.step(n_every)
        steps += n_every
        d = grid.diagnostics(profiles=True)
        cw = centre_and_width(d["phi_avg"].cpu().numpy(), band_sign)
        if cw is None:
            rows.append((steps * dt, math.nan, math.nan, math.nan))
        else:
            rows.append((steps * dt, cw[0], cw[1], laplace_pressure(d["p_avg"].cpu().numpy(), cw[0])))
    return tuple(np.array(c) for c in zip(*rows))
