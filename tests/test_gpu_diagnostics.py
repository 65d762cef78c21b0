"""GPU diagnostics against the oracle, and the FP32-vs-FP64 precision study on the spinodal
coarsening workload (the precision growth direction: mass, phi and the coarsening length
L_d(t) = A_total / L_I(t) of section IV)."""
import math

import numpy as np
import pytest

from paper_1904_10070_amd import inputs
from tests.helpers import oracle_run

pytestmark = pytest.mark.gpu


def test_diagnostics_match_oracle_fp64(torch_cuda):
    from paper_1904_10070_amd import TorusGrid
    p = inputs.drop_workload()
    phi = inputs.drop_workload_phi(p, seed=1)
    n, ut, up = inputs.rest_moments(p.n_theta, p.n_phi)
    og, _, _ = oracle_run(p, phi, n, ut, up, 200)
    g = TorusGrid(p, precision=64)
    g.set_state(phi, n, ut, up)
    g.step(200)
    dg, do = g.diagnostics(), og.diagnostics()
    assert abs(dg["L_I"] - do["L_I"]) <= 1e-12 * do["L_I"]
    assert abs(dg["A_total"] - do["A_total"]) <= 1e-13 * do["A_total"]
    assert np.abs(dg["phi_avg"].cpu().numpy() - do["phi_avg"]).max() <= 1e-12
    assert np.abs(dg["p_avg"].cpu().numpy() - do["p_avg"]).max() <= 1e-12
    assert abs(do["A_total"] - 4 * math.pi ** 2 * p.r * p.R) < 1e-11


@pytest.mark.parametrize("shape,precision", [((24, 80), 64), ((37, 150), 64), ((512, 1280), 64),
                                             ((512, 1280), 32), ((33, 7), 32)])
def test_structure_length_matches_oracle(torch_cuda, shape, precision):
    """The direct FP64 DFT of the library against numpy's FFT (oracle/structure.py) on seeded
    fields; FP32 grids hold phi rounded to FP32, which the reference receives too."""
    from paper_1904_10070_amd import TorusGrid
    from oracle import structure
    p = inputs.TorusParams(1.0, 2.5, shape[0], shape[1], 0.5, 2e-3, 0.05, 0.3, 2e-4)
    phi = inputs.spinodal_phi(p, seed=11) + 0.3 * np.sin(
        2 * np.pi * np.arange(shape[0]) / shape[0] * 3)[:, None]
    g = TorusGrid(p, precision)
    g.set_state(phi, *inputs.rest_moments(*shape))
    got = g.structure_length()
    ref = structure.structure_length(phi if precision == 64 else phi.astype(np.float32), 1.0, 2.5)
    print(f"{shape} FP{precision}: L_S {got[0]:.6f} reference {ref[0]:.6f}", flush=True)
    for a, b in zip(got, ref):
        assert abs(a - b) <= 1e-10 * abs(b), (a, b)


@pytest.mark.parametrize("tau", [0.6, 2.0])
def test_spinodal_fp32_against_fp64(torch_cuda, tau):
    """512 x 1280 spinodal workload, 50,000 steps (t = 20) in both precisions from the same
    seeded phi: L_d(t) and the structure-factor length L_S(t) agree within 2 % once domains
    have formed (t >= 6) (L_d measured 4e-4).
    Mass: FP64 drifts by less than 1e-11; FP32, which stores deviations from the rest
    equilibrium, by 8e-8 (bar 1e-6; plain FP32 storage drifted by 1.8e-3)."""
    from paper_1904_10070_amd import TorusGrid
    p = inputs.spinodal_workload(tau)
    phi = inputs.spinodal_phi(p, seed=7)
    n, ut, up = inputs.rest_moments(p.n_theta, p.n_phi)
    grids = {}
    for prec in (64, 32):
        g = TorusGrid(p, precision=prec)
        g.set_state(phi, n, ut, up)
        grids[prec] = g
    m0 = grids[64].invariants()[0]
    every, total = 2500, 50000
    rows = []
    for it in range(every, total + 1, every):
        for g in grids.values():
            g.step(every)
        L = {prec: g.diagnostics(profiles=False)["L_d"] for prec, g in grids.items()}
        LS = {prec: g.structure_length()[0] for prec, g in grids.items()}
        rows.append((it * p.dt, L[64], L[32], LS[64], LS[32]))
    t, l64, l32, s64, s32 = (np.array(x) for x in zip(*rows))
    rel = np.abs(l32 - l64) / l64
    rel_s = np.abs(s32 - s64) / s64
    drift = {prec: abs(g.invariants()[0] - m0) / m0 for prec, g in grids.items()}
    print(f"tau={tau}: L_d(t=20) fp64 {l64[-1]:.4f} fp32 {l32[-1]:.4f}; max rel diff t>=6 "
          f"{rel[t >= 6].max():.3e}; L_S(t=20) fp64 {s64[-1]:.4f} fp32 {s32[-1]:.4f}, max rel "
          f"diff t>=6 {rel_s[t >= 6].max():.3e}; mass drift fp64 {drift[64]:.2e} fp32 "
          f"{drift[32]:.2e}", flush=True)
    assert np.all(np.diff(l64[t >= 6]) > -0.05 * l64[t >= 6][:-1])   # coarsening, L_d grows
    assert np.all(np.diff(s64[t >= 6]) > -0.05 * s64[t >= 6][:-1])   # and L_S
    assert rel[t >= 6].max() <= 0.02 and rel_s[t >= 6].max() <= 0.02
    assert drift[64] < 1e-11 and drift[32] < 1e-6
