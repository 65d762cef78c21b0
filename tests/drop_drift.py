"""Drops on a torus drift to the outer equator (section III D of the paper), on the GPU.

TEST INFRASTRUCTURE: used by test_gpu_drift.py, and run as
`python -m tests.drop_drift [64|32] [t_end]` from the repository root for the paper's length.

Set-up (the paper's): r = 0.8, R = 2, kappa = 5e-4, A = 0.5, tau = M = 2.5e-3, dt = 5e-4, on a
256 x 640 grid (the paper does not give its grid); drops by eq. drop_init (phi = -1 inside)
at (theta_0, phi_0 = 0) with the printed (theta_0, R_0) pairs, which give them about the area
of a drop of radius 30 xi_0 on the outer equator.  The three drops run as one ensemble; the
centre theta_c is the polar angle of the area-weighted centroid of the drop's phase, from the
GPU's azimuthal average <phi>(theta).
"""
import math
import sys

import numpy as np

from paper_1904_10070_amd import inputs

DROPS = ((0.5, 0.938), (0.7, 0.924), (0.9, 0.910))   # theta_0 / pi, R_0 (section III D)
PARAMS = inputs.TorusParams(0.8, 2.0, 256, 640, 0.5, 5e-4, 2.5e-3, 2.5e-3, 5e-4)


def signed(theta):
    """Angle in (-pi, pi]."""
    return (np.asarray(theta) + math.pi) % (2 * math.pi) - math.pi


def run(precision, t_end, every_t=1.0, progress=None):
    """(t, [signed theta_c(t) of each drop], [relative mass drift of each drop])."""
    from paper_1904_10070_amd import TorusGrid, TorusBatch, stripe
    p = PARAMS
    grids = []
    for th0, R0 in DROPS:
        g = TorusGrid(p, precision)
        g.set_state(inputs.drop_phi(p, th0 * math.pi, 0.0, R0),
                    *inputs.rest_moments(p.n_theta, p.n_phi))
        grids.append(g)
    m0 = [g.invariants()[0] for g in grids]
    batch = TorusBatch(grids)
    t, recs = stripe.record(batch.step, grids, t_end, every_t, stripe.drop_state, progress)
    drift = [abs(g.invariants()[0] - m) / m for g, m in zip(grids, m0)]
    batch.close()
    for g in grids:
        g.close()
    return t, [signed(c) for c in recs], drift


def main(argv):
    prec = int(argv[1]) if len(argv) > 1 else 32
    t_end = float(argv[2]) if len(argv) > 2 else 1800.0
    t, tracks, drift = run(prec, t_end, progress=lambda x: print(f"  t = {x:.0f}", flush=True))
    print(f"FP{prec}, t_end = {t_end:g}, largest mass drift {max(drift):.1e}")
    every = max(1, int(round(25.0 / (t[1] - t[0]))))
    print("| t | " + " | ".join(f"theta_0 = {th0} pi" for th0, _ in DROPS) + " |")
    print("|---|" + "---|" * len(DROPS))
    for i in range(0, len(t), every):
        print(f"| {t[i]:.0f} | " + " | ".join(f"{s[i] / math.pi:+.4f} pi" for s in tracks) + " |")


if __name__ == "__main__":
    main(sys.argv)
