"""Damped oscillation of stripes about their equilibrium on the GPU, against the closed forms
of section III C of the paper (eqs. stripe_hydro_sol, stripe_alphanu, stripe_hydro_omega0_pi
and stripe_hydro_omega0_npi).

TEST INFRASTRUCTURE (imports the oracle's closed forms and fits): used by test_gpu_drift.py
for a reduced set, and run as `python -m tests.stripe_sweep [64|32] [t_end]` from the
repository root for the whole sweep of the paper's set-up:

  tori with a = r / R = 0.4: r = 0.8, 1, 1.2 on N_theta = 320, 400, 480 nodes (N_phi = 64: the
  stripes do not depend on phi); A = 0.5, M = nu, dt = 5e-4; a stripe (the phi = -1 phase,
  eq. stripe_tanh with its offset) started pi/20 away from equilibrium: theta_0 = 0.95 pi with
  width 0.28 pi (equilibrium at pi) or theta_0 = 0.7 pi with width 0.786 pi (equilibrium at
  3 pi / 4); nu = 2.5e-3, 5e-3, 7.5e-3 at kappa = 5e-4, and kappa = 2.5e-4, 6.25e-4 at
  nu = 2.5e-3.

All tori of one precision run as one ensemble (one launch per Runge-Kutta stage).  The centre
theta_c(t) is measured every time unit from the GPU's azimuthal average <phi>(theta); the fit
is eq. stripe_hydro_sol with omega and alpha free and the phase zero, as in the paper, and,
beside it, with phase and offset free as well.
"""
import math
import sys

import numpy as np

from oracle import stripe_theory as st
from paper_1904_10070_amd import inputs

GEOMETRIES = ((0.8, 320), (1.0, 400), (1.2, 480))      # (r, N_theta), R = r / 0.4
CASES = {"pi": (0.95, 0.28), "3pi/4": (0.7, 0.786)}     # theta_0 / pi, width / pi
NU_SET = (2.5e-3, 5e-3, 7.5e-3)                         # at kappa = 5e-4
KAPPA_SET = (2.5e-4, 6.25e-4)                           # at nu = 2.5e-3
N_PHI = 64
DT = 5e-4


CH4 = 32  # the fourth-order Cahn-Hilliard variant (include/tlb.h)


def torus(r, n_theta, nu, kappa=5e-4, M=None, dt=DT, flags=0):
    """A torus of the sweep: R = r / 0.4, A = 0.5, M = nu unless given."""
    return inputs.TorusParams(r, r / 0.4, n_theta, N_PHI, 0.5, kappa, nu if M is None else M,
                              nu, dt, flags)


def configs(geometries=GEOMETRIES, cases=tuple(CASES), nus=NU_SET, kappas=KAPPA_SET, flags=0):
    """(case, TorusParams) of the sweep."""
    out = []
    for r, nt in geometries:
        for case in cases:
            for nu, kappa in [(nu, 5e-4) for nu in nus] + [(2.5e-3, k) for k in kappas]:
                out.append((case, torus(r, nt, nu, kappa, flags=flags)))
    return out


def run(cfgs, precision, t_end, every_t=1.0, progress=None):
    """Run the configurations as one ensemble; one result dict per configuration."""
    from paper_1904_10070_amd import TorusGrid, TorusBatch, stripe
    import torch
    # grids stepped one by one (no batch) each get a stream of their own, so that the small
    # grids' kernels run side by side
    own_streams = any(p.flags & CH4 for _, p in cfgs)
    grids = []
    for case, p in cfgs:
        th0, w0 = CASES[case]
        g = TorusGrid(p, precision, stream=torch.cuda.Stream() if own_streams else None)
        g.set_state(inputs.stripe_phi(p, th0 * math.pi, w0 * math.pi),
                    *inputs.rest_moments(p.n_theta, p.n_phi))
        grids.append(g)
    m0 = [g.invariants()[0] for g in grids]
    if any(p.flags & CH4 for _, p in cfgs):  # no batches for the fourth-order variant
        batch = None

        def step(k):
            for g in grids:
                g.step(k)
    else:
        batch = TorusBatch(grids)
        step = batch.step
    t, recs = stripe.record(step, grids, t_end, every_t,
                            lambda g: stripe.stripe_state(g, band_sign=-1.0), progress)
    out = []
    for (case, p), g, rec, m in zip(cfgs, grids, recs, m0):
        rec = np.array(rec)
        res = analyse(case, p, t, rec[:, 0], rec[:, 1])
        res["mass_drift"] = abs(g.invariants()[0] - m) / m
        res["flags"] = p.flags
        out.append(res)
    if batch is not None:
        batch.close()
    for g in grids:
        g.close()
    return out


def analyse(case, p, t, centre, width):
    """Fits of eq. stripe_hydro_sol to theta_c(t) - theta_c^eq and the closed forms."""
    th0, w0 = CASES[case]
    pred = st.predict(p.gamma, p.r, p.R, 1.0, p.tau, th0 * math.pi, w0 * math.pi)
    eq = min(pred, key=lambda x: abs(x["theta_c"] - centre[-1]))
    dth = centre - eq["theta_c"]
    w_fit, a_fit = st.fit_damped_oscillation(t, dth, dth[0])
    w_free, a_free = st.fit_damped_oscillation_window(t, dth, eq["omega0"], eq["alpha"], 0.0)
    return dict(case=case, r=p.r, R=p.R, n_theta=p.n_theta, nu=p.tau, M=p.M, kappa=p.kappa,
                theta_eq=eq["theta_c"], width_eq=eq["dtheta"], omega0=eq["omega0"],
                alpha_nu=eq["alpha"], omega_fit=w_fit, alpha_fit=a_fit, omega_free=w_free,
                alpha_free=a_free, theta_end=float(centre[-1]), width_end=float(width[-1]),
                finite=bool(np.all(np.isfinite(centre))))


def table(rows):
    head = ("| case | CH order | r | N_theta | nu | M | kappa | omega_0 | omega fit | alpha_nu | "
            "alpha fit | omega / alpha (phase, offset free) | theta_c end - eq |")
    lines = [head, "|" + "---|" * 13]
    for x in rows:
        lines.append(
            f"| {x['case']} | {4 if x.get('flags', 0) & CH4 else 2} | {x['r']} | {x['n_theta']} | "
            f"{x['nu']:.2e} | {x['M']:.2e} | "
            f"{x['kappa']:.2e} | {x['omega0']:.5f} | "
            f"{x['omega_fit']:.5f} ({x['omega_fit'] / x['omega0'] - 1:+.1%}) | "
            f"{x['alpha_nu']:.2e} | {x['alpha_fit']:.2e} ({x['alpha_fit'] / x['alpha_nu']:.2f}x) | "
            f"{x['omega_free']:.5f} / {x['alpha_free']:.2e} | "
            f"{(x['theta_end'] - x['theta_eq']) / math.pi:+.4f} pi |")
    return "\n".join(lines)


def main(argv):
    prec = int(argv[1]) if len(argv) > 1 else 64
    t_end = float(argv[2]) if len(argv) > 2 else 800.0
    if len(argv) > 3 and argv[3] == "ch4":
        # the second- against the fourth-order Cahn-Hilliard discretisation on the r = 0.8
        # torus, N_theta = 320 unless given (nu sweep at kappa = 5e-4)
        nt = int(argv[4]) if len(argv) > 4 else 320
        # finer grids: the time step scaled with the square of the spacing (the explicit
        # Cahn-Hilliard bound; the fourth-order operator's spectrum is larger) and the two ends
        # of the viscosity range
        scale = (320.0 / nt) ** 2 if nt > 320 else 1.0
        nus = NU_SET if nt <= 320 else (NU_SET[0], NU_SET[-1])
        cfgs = [(c, p.with_(flags=fl, dt=p.dt * scale)) for fl in (0, CH4)
                for c, p in configs(geometries=((0.8, nt),), nus=nus, kappas=())]
    else:
        cfgs = configs()
    rows = run(cfgs, prec, t_end, progress=lambda t: print(f"  t = {t:.0f}", flush=True))
    print(f"FP{prec}, t_end = {t_end:g}")
    print(table(rows))
    print("largest mass drift", max(x["mass_drift"] for x in rows))


if __name__ == "__main__":
    main(sys.argv)
