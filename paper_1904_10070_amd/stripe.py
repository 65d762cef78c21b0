"""Stripe and drop measurements from the GPU diagnostics (section III of the paper): the band's
centre theta_c and angular width from the azimuthal average <phi>(theta) (eq. phiavg), the
Laplace pressure as the difference of the azimuthally averaged pressure
p = n + A(-phi^2/2 + 3 phi^4/4) (eq. pbin) across the torus, at the node nearest theta_c and
the node opposite it (theta_c + pi), and a drop's centre theta_c as the polar angle of the
area-weighted centroid of its phase (section III D).  The profiles come from tlb_diagnostics;
only the searches and sums over n_theta host values run here.
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


def drop_centre(phi_avg, r, R, drop_sign=-1.0):
    """theta of the centroid of the phase drop_sign * phi > 0 on the circle of polar angles,
    weighted by the area element (R + r cos theta) and the local fraction (1 + drop_sign *
    <phi>) / 2 of that phase at each theta."""
    prof = np.asarray(phi_avg, dtype=np.float64)
    nt = prof.size
    th = np.arange(nt) * (2.0 * math.pi / nt)
    w = (R + r * np.cos(th)) * (1.0 + drop_sign * prof) * 0.5
    z = np.sum(w * np.exp(1j * th))
    return math.atan2(z.imag, z.real) % (2.0 * math.pi)


def record(step, grids, t_end, every_t, measure, progress=None):
    """Advance with step(n) (a TorusGrid's or a TorusBatch's step) to t_end, applying
    measure(grid) to every grid every every_t of simulated time, the first time at t = 0.  All
    grids share one time step.  Returns (times, [measurements of grid 0, of grid 1, ...]);
    progress(t) is called every 100 records if given."""
    dt = grids[0].params.dt
    assert all(abs(g.params.dt - dt) <= 1e-15 * dt for g in grids), "grids with different dt"
    n_every = int(round(every_t / dt))
    ts, out = [], [[] for _ in grids]
    steps = 0
    while True:
        ts.append(steps * dt)
        for g, o in zip(grids, out):
            o.append(measure(g))
        if progress is not None and len(ts) % 100 == 0:
            progress(ts[-1])
        if steps * dt >= t_end - 0.5 * dt:
            break
        step(n_every)
        steps += n_every
    return np.array(ts), out


def stripe_state(grid, band_sign=1.0):
    """(theta_c, width, Laplace pressure) of the band of a grid, NaN where none is found."""
    d = grid.diagnostics(profiles=True)
    cw = centre_and_width(d["phi_avg"].cpu().numpy(), band_sign)
    if cw is None:
        return math.nan, math.nan, math.nan
    return cw[0], cw[1], laplace_pressure(d["p_avg"].cpu().numpy(), cw[0])


def drop_state(grid, drop_sign=-1.0):
    """theta_c of the drop of a grid (drop_centre of its <phi>(theta))."""
    d = grid.diagnostics(profiles=True)
    return drop_centre(d["phi_avg"].cpu().numpy(), grid.params.r, grid.params.R, drop_sign)


def track_drop(grid, t_end, every_t, drop_sign=-1.0, progress=None):
    """(t, theta_c) of the drop of one grid every every_t up to t_end, from t = 0."""
    t, (c,) = record(grid.step, [grid], t_end, every_t, lambda g: drop_state(g, drop_sign),
                     progress)
    return t, np.array(c)


def track(grid, t_end, every_t, band_sign=1.0):
    """Advance `grid` (a TorusGrid) to t_end, recording (t, theta_c, width, dp) every every_t
    of simulated time, the first record after every_t.  Returns four numpy arrays (NaN where
    the band is not found)."""
    t, (rows,) = record(grid.step, [grid], t_end, every_t, lambda g: stripe_state(g, band_sign))
    rows = np.array(rows)
    return t[1:], rows[1:, 0], rows[1:, 1], rows[1:, 2]
