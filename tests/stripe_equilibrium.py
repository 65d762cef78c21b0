"""Where stripes come to rest, and their Laplace pressure there, on the GPU (section III A and B
of the paper: the equilibrium positions of Fig. tor_stripe_fork and the Laplace pressure test
of Fig. stripe_laplace).

TEST INFRASTRUCTURE (imports the oracle's closed forms): run as
`python -m tests.stripe_equilibrium [fork|laplace] [64|32] [t_end] [N_theta (fork)]` from the
repository root.

Common set-up (the paper's): r = 0.8, R = 2, N_theta = 320 (N_phi = 64: the stripes do not
depend on phi), A = 0.5, nu = M = 2.5e-3, dt = 5e-4, the stripe is the phi = -1 phase
(eq. stripe_tanh with its offset).  All stripes of one run form one ensemble.

fork: widths 0.95, 0.65, 0.6 and 0.3 pi started at theta_0 = pi / 2 (kappa = 5e-4).  The paper
  finds them at rest on the upper side (theta_c < pi), the lower side, the upper side, and at
  pi: the larger stripes have two equilibria, pi -/+ arccos(cos(dtheta_eq / 2) / a), and which
  one traps the stripe depends on how often its centre crosses pi while the oscillation decays.
laplace: stripes of area ratio dA / dA_crit from 0.3 to 1.9, for kappa = 2.5e-4 and 5e-4,
  started 0.05 pi above their (upper) equilibrium; at the end the measured pressure difference
  (mean over the last tenth of the run) against eq. stripe_laplace_eq.
"""
import math
import sys

import numpy as np
from scipy.optimize import brentq

from oracle import stripe_theory as st
from paper_1904_10070_amd import inputs

BASE = dict(r=0.8, R=2.0, n_theta=320, n_phi=64, A=0.5, kappa=5e-4, M=2.5e-3, tau=2.5e-3,
            dt=5e-4)
FORK_WIDTHS = (0.95, 0.65, 0.6, 0.3)                    # / pi, started at theta_0 = pi / 2
FORK_PAPER = ("upper", "lower", "upper", "pi")          # where the paper finds them at rest
AREA_RATIOS = (0.3, 0.5, 0.7, 0.9, 1.1, 1.3, 1.6, 1.9)
KAPPAS = (2.5e-4, 5e-4)


def side(theta_c, tol=0.01 * math.pi):
    if abs(theta_c - math.pi) <= tol:
        return "pi"
    return "upper" if theta_c < math.pi else "lower"


def crossings(centre):
    """Number of times theta_c(t) crosses pi."""
    s = np.sign(np.asarray(centre) - math.pi)
    s = s[s != 0]
    return int(np.count_nonzero(s[1:] != s[:-1]))


def run_ensemble(starts, precision, t_end, every_t=1.0, progress=None):
    """starts: list of (TorusParams, theta_0, width_0).  Returns t and, per stripe, the rows
    (theta_c, width, dp) of every record, and the relative mass drifts."""
    from paper_1904_10070_amd import TorusGrid, TorusBatch, stripe
    import torch
    # grids stepped one by one (no batch) each get a stream of their own, so that the small
    # grids' kernels run side by side
    own_streams = any(p.flags & CH4 for p, _, _ in starts)
    grids = []
    for p, th0, w0 in starts:
        g = TorusGrid(p, precision, stream=torch.cuda.Stream() if own_streams else None)
        g.set_state(inputs.stripe_phi(p, th0, w0), *inputs.rest_moments(p.n_theta, p.n_phi))
        grids.append(g)
    m0 = [g.invariants()[0] for g in grids]
    if any(p.flags & CH4 for p, _, _ in starts):  # no batches for the fourth-order variant
        batch = None

        def step(k):
            for g in grids:
                g.step(k)
    else:
        batch = TorusBatch(grids)
        step = batch.step
    t, recs = stripe.record(step, grids, t_end, every_t,
                            lambda g: stripe.stripe_state(g, band_sign=-1.0), progress)
    drift = [abs(g.invariants()[0] - m) / m for g, m in zip(grids, m0)]
    if batch is not None:
        batch.close()
    for g in grids:
        g.close()
    return t, [np.array(r) for r in recs], drift


CH4 = 32  # the fourth-order Cahn-Hilliard variant (include/tlb.h)


def fork(precision=64, t_end=3000.0, progress=None, n_theta=320, flags=0):
    p = inputs.TorusParams(**dict(BASE, n_theta=n_theta), flags=flags)
    starts = [(p, 0.5 * math.pi, w * math.pi) for w in FORK_WIDTHS]
    t, recs, drift = run_ensemble(starts, precision, t_end, progress=progress)
    rows = []
    for w, paper, rec, d in zip(FORK_WIDTHS, FORK_PAPER, recs, drift):
        area = st.stripe_area(p.r, p.R, 0.5 * math.pi, w * math.pi)
        eqs = st.equilibria(p.r, p.R, area)
        c = rec[:, 0]
        nearest = min(eqs, key=lambda e: abs(e[0] - c[-1]))
        rows.append(dict(width0=w, area_ratio=area / st.critical_area(p.r, p.R), paper=paper,
                         side=side(c[-1]), crossings=crossings(c), theta_end=float(c[-1]),
                         theta_eq=nearest[0], width_end=float(rec[-1, 1]), width_eq=nearest[1],
                         last_crossing=float(t[np.nonzero(np.diff(np.sign(c - math.pi)))[0][-1]])
                         if crossings(c) else 0.0, mass_drift=d, centre=c))
    return t, rows


def laplace_starts():
    out = []
    for kappa in KAPPAS:
        p = inputs.TorusParams(**dict(BASE, kappa=kappa))
        crit = st.critical_area(p.r, p.R)
        for ratio in AREA_RATIOS:
            tc, dth = st.equilibria(p.r, p.R, ratio * crit)[0]
            th0 = tc - 0.05 * math.pi
            w0 = brentq(lambda d: st.stripe_area(p.r, p.R, th0, d) - ratio * crit, 1e-6,
                        2 * math.pi - 1e-6)
            out.append((p, th0, w0))
    return out


def laplace(precision=64, t_end=2000.0, progress=None):
    starts = laplace_starts()
    t, recs, drift = run_ensemble(starts, precision, t_end, progress=progress)
    late = t >= 0.9 * t_end
    rows = []
    for (p, th0, w0), rec, d in zip(starts, recs, drift):
        area = st.stripe_area(p.r, p.R, th0, w0)
        tc, dth = min(st.equilibria(p.r, p.R, area), key=lambda e: abs(e[0] - rec[-1, 0]))
        dp_eq = st.laplace_pressure(p.gamma, p.r, p.R, tc, dth)
        rows.append(dict(kappa=p.kappa, area_ratio=area / st.critical_area(p.r, p.R),
                         theta_eq=tc, width_eq=dth, dp_eq=dp_eq,
                         theta_end=float(rec[late, 0].mean()),
                         width_end=float(rec[late, 1].mean()), dp=float(rec[late, 2].mean()),
                         dp_sd=float(rec[late, 2].std()), mass_drift=d))
    return rows


def main(argv):
    what = argv[1] if len(argv) > 1 else "fork"
    prec = int(argv[2]) if len(argv) > 2 else 64
    prog = lambda t: print(f"  t = {t:.0f}", flush=True)
    if what == "fork":
        t_end = float(argv[3]) if len(argv) > 3 else 3000.0
        n_theta = int(argv[4]) if len(argv) > 4 else 320
        flags = CH4 if len(argv) > 5 and argv[5] == "ch4" else 0
        t, rows = fork(prec, t_end, prog, n_theta, flags)
        print(f"FP{prec}, N_theta = {n_theta}, t_end = {t_end:g}, "
              f"Cahn-Hilliard order {4 if flags else 2}")
        print("| width_0 | dA / dA_crit | paper | here | crossings of pi | last crossing | "
              "theta_c end | theta_eq | width end | width_eq |")
        print("|" + "---|" * 10)
        for x in rows:
            print(f"| {x['width0']} pi | {x['area_ratio']:.2f} | {x['paper']} | {x['side']} | "
                  f"{x['crossings']} | {x['last_crossing']:.0f} | "
                  f"{x['theta_end'] / math.pi:.4f} pi | {x['theta_eq'] / math.pi:.4f} pi | "
                  f"{x['width_end'] / math.pi:.4f} pi | {x['width_eq'] / math.pi:.4f} pi |")
        print("largest mass drift", max(x["mass_drift"] for x in rows))
        for x in rows:
            print(f"centre / pi every 50, width {x['width0']}: " +
                  " ".join(f"{c / math.pi:.3f}" for c in x["centre"][::50]))
    else:
        t_end = float(argv[3]) if len(argv) > 3 else 2000.0
        rows = laplace(prec, t_end, prog)
        print(f"FP{prec}, t_end = {t_end:g}")
        print("| kappa | dA / dA_crit | theta_eq | theta_c (end) | width_eq | width (end) | "
              "dp eq. stripe_laplace_eq | dp measured | ratio | sd |")
        print("|" + "---|" * 10)
        for x in rows:
            print(f"| {x['kappa']:.2e} | {x['area_ratio']:.2f} | {x['theta_eq'] / math.pi:.4f} pi | "
                  f"{x['theta_end'] / math.pi:.4f} pi | {x['width_eq'] / math.pi:.4f} pi | "
                  f"{x['width_end'] / math.pi:.4f} pi | {x['dp_eq']:.4e} | {x['dp']:.4e} | "
                  f"{x['dp'] / x['dp_eq']:.4f} | {x['dp_sd']:.1e} |")
        print("largest mass drift", max(x["mass_drift"] for x in rows))


if __name__ == "__main__":
    main(sys.argv)
