"""Coarsening of an even mixture on a torus on the GPU (section IV B of the paper, Fig.
tscal-ev): the domain length L_d = A_total / L_I grows with an apparent exponent of 2/3 with
hydrodynamics (viscous-inertial regime) and 1/3 without the convective term of the
Cahn-Hilliard equation (diffusive regime), until the domains wrap round the tube.

TEST INFRASTRUCTURE (a study script beside the tests): run as
`python -m tests.coarsening [hydro|diffusive] [64|32] [t_end]` from the repository root.

Set-up (the paper's): R = 2.5, r = 1, N_theta x N_phi = 400 x 800, phi = uniform noise in
(-0.1, 0.1) about 0 (eq. phirand; seed 7), n = 20 at rest, A = 0.5, kappa = 5e-4,
tau = M = 2.5e-3, dt = 5e-4.  L_d and the structure-factor length L_S are taken on the GPU at
logarithmically spaced times; the exponent is the least-squares slope of log L against log t
over a window.
"""
import sys

import numpy as np

from paper_1904_10070_amd import inputs

PARAMS = inputs.TorusParams(1.0, 2.5, 400, 800, 0.5, 5e-4, 2.5e-3, 2.5e-3, 5e-4)
N0 = 20.0
WINDOWS = {"hydro": (40.0, 250.0), "diffusive": (350.0, 3000.0)}


def sample_steps(t_end, dt, n=60, t_first=1.0):
    """Step counts at about n logarithmically spaced times from t_first to t_end."""
    ts = np.geomspace(t_first, t_end, n)
    return sorted({int(round(t / dt)) for t in ts})


def run(mode, precision, t_end, seed=7, progress=None):
    """(t, L_d, L_S, relative mass drift) of one run; mode 'hydro' or 'diffusive'."""
    from paper_1904_10070_amd import CH_NO_ADVECTION, TorusGrid
    p = PARAMS.with_(flags=CH_NO_ADVECTION if mode == "diffusive" else 0)
    g = TorusGrid(p, precision)
    g.set_state(inputs.spinodal_phi(p, seed), *inputs.rest_moments(p.n_theta, p.n_phi, N0))
    m0 = g.invariants()[0]
    done = 0
    ts, Ld, LS = [], [], []
    for k in sample_steps(t_end, p.dt):
        g.step(k - done)
        done = k
        ts.append(k * p.dt)
        Ld.append(g.diagnostics(profiles=False)["L_d"])
        LS.append(g.structure_length()[0])
        if progress is not None:
            progress(ts[-1], Ld[-1])
    inv = g.invariants()
    g.close()
    assert inv[2] == 0, "non-finite values"
    return np.array(ts), np.array(Ld), np.array(LS), abs(inv[0] - m0) / m0


def exponent(t, L, t0, t1):
    """Slope of log L against log t for t0 <= t <= t1."""
    m = (t >= t0) & (t <= t1)
    return float(np.polyfit(np.log(t[m]), np.log(L[m]), 1)[0])


def main(argv):
    mode = argv[1] if len(argv) > 1 else "hydro"
    prec = int(argv[2]) if len(argv) > 2 else 32
    t_end = float(argv[3]) if len(argv) > 3 else (500.0 if mode == "hydro" else 3000.0)
    t, Ld, LS, drift = run(mode, prec, t_end,
                           progress=lambda x, l: print(f"  t = {x:.1f} L_d = {l:.4f}", flush=True))
    t0, t1 = WINDOWS[mode]
    print(f"{mode} FP{prec}, t_end = {t_end:g}, mass drift {drift:.1e}")
    print(f"apparent exponent over t in [{t0:g}, {min(t1, t_end):g}]: L_d {exponent(t, Ld, t0, t1):.3f}, "
          f"L_S {exponent(t, LS, t0, t1):.3f}")
    print("| t | L_d | L_S |")
    print("|---|---|---|")
    for x, a, b in zip(t, Ld, LS):
        print(f"| {x:.1f} | {a:.4f} | {b:.4f} |")


if __name__ == "__main__":
    main(sys.argv)
