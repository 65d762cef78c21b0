"""GPU parity: the HIP library (through its C interface) against the CPU oracle.

Both sides start from the same host arrays built by paper_1904_10070_amd.inputs and set their
own equilibrium populations.  Bars:
  * FP64: relative L-infinity error <= 1e-12 on f, phi, n and mu, conservation sums within
    1e-13 of the oracle's.  The velocity u = sum_k f_k v_k / n is a sum that cancels to |u|
    much smaller than its terms in a slow flow, so its error is measured, as that of any
    computed sum, relative to the magnitude of the terms it adds: |du|_inf <= 1e-12 times
    max over nodes of sum_k |f_k v_k| / n (see velocity_scale);
  * FP32 (against the FP64 oracle): about ten times the error of the same oracle source run in
    FP32 on the CPU -- on the 64 x 160 drop workload after 2000 steps that envelope is
    f 1.1e-4, phi 5.7e-5, n 9.4e-5, u 2.3e-3, mass 2.3e-5 -- so the bars are
    f, n <= 1.5e-3, phi <= 1e-3, u <= 3e-2, mass <= 3e-4.
"""
import math

import numpy as np
import pytest

from paper_1904_10070_amd import inputs
from tests.helpers import rel_linf, oracle_run, gpu_run, velocity_scale

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def moments_np(m):
    return {k: (v.double().cpu().numpy() if v is not None else None) for k, v in m.items()}


def compare_fp64(p, phi, n, ut, up, steps, tol=FP64_TOL, flags_note=""):
    og, f_ref, phi_ref = oracle_run(p, phi, n, ut, up, steps)
    gg, f_gpu, phi_gpu = gpu_run(p, phi, n, ut, up, steps)
    ef, ep = rel_linf(f_gpu, f_ref), rel_linf(phi_gpu, phi_ref)
    mr = og.moments()
    mg = moments_np(gg.moments())
    errs = {"f": ef, "phi": ep}
    for k in ("n", "mu"):
        errs[k] = rel_linf(mg[k], mr[k])
    for axis, k in enumerate(("u_theta", "u_phi")):
        errs[k] = float(np.abs(mg[k] - mr[k]).max()) / velocity_scale(f_ref, mr["n"], axis)
    print(f"{p.n_theta}x{p.n_phi} {flags_note} steps={steps}", {k: f"{v:.2e}" for k, v in errs.items()},
          flush=True)
    for k, v in errs.items():
        assert v <= tol, (k, v)
    return og, gg


def test_drop_workload_fp64_2000_steps(torch_cuda):
    """64 x 160 torus, one drop near theta = pi/2, 2000 steps (t = 1)."""
    p = inputs.drop_workload()
    phi = inputs.drop_workload_phi(p, seed=1)
    n, ut, up = inputs.rest_moments(p.n_theta, p.n_phi)
    og, gg = compare_fp64(p, phi, n, ut, up, 2000)
    mo, so, bo = og.invariants()
    mg, sg, bg = gg.invariants()
    assert bo == 0 and bg == 0
    assert abs(mg - mo) <= 1e-13 * abs(mo)
    assert abs(sg - so) <= 1e-13 * abs(mo)


@pytest.mark.parametrize("shape", [(37, 150), (9, 70), (4, 64), (6, 1), (3, 5), (1, 9), (66, 130)])
def test_random_state_ragged_fp64(torch_cuda, shape):
    """Away from equilibrium, on grids with ragged tiles and wrap-around halos."""
    nt, np_ = shape
    p = inputs.TorusParams(1.0, 2.5, nt, np_, 0.5, 2e-3, 0.05, 0.3, 2e-4)
    phi, n, ut, up = inputs.random_state(p, seed=nt * 1000 + np_)
    compare_fp64(p, phi, n, ut, up, 25)


@pytest.mark.parametrize("flags", [inputs_flag for inputs_flag in (1, 2, 3)])
def test_flag_variants_fp64(torch_cuda, flags):
    """Flat limit (J = R, G = 0) and the Cahn-Hilliard equation without advection."""
    p = inputs.TorusParams(1.0, 2.5, 24, 96, 0.5, 2e-3, 0.05, 0.3, 2e-4, flags)
    phi, n, ut, up = inputs.random_state(p, seed=11 + flags)
    compare_fp64(p, phi, n, ut, up, 25, flags_note=f"flags={flags}")


def test_stripe_gpu_2d_equals_oracle_1d(torch_cuda):
    """A phi-independent stripe stays phi-independent: the GPU at 256 x 640 against the oracle
    at 256 x 1 (the stripe workload, R = 2, band of full width 0.3 pi)."""
    p2 = inputs.stripe_workload(R=2.0, n_theta=256, n_phi=640)
    p1 = p2.with_(n_phi=1)
    theta0 = 2 * math.pi * np.random.default_rng(2).uniform()
    phi1 = inputs.stripe_phi(p1, theta0, 0.3 * math.pi, sign=-1.0)
    phi2 = np.repeat(phi1, p2.n_phi, axis=1)
    steps = 400
    _, f_ref, phi_ref = oracle_run(p1, phi1, *inputs.rest_moments(256, 1), steps)
    _, f_gpu, phi_gpu = gpu_run(p2, phi2, *inputs.rest_moments(256, 640), steps)
    spread = np.abs(phi_gpu - phi_gpu[:, :1]).max()
    assert spread <= 1e-13, spread
    assert rel_linf(phi_gpu, np.repeat(phi_ref, 640, axis=1)) <= FP64_TOL
    assert rel_linf(f_gpu, np.repeat(f_ref, 640, axis=2)) <= FP64_TOL


def test_drop_workload_fp32_tolerance(torch_cuda):
    p = inputs.drop_workload()
    phi = inputs.drop_workload_phi(p, seed=1)
    n, ut, up = inputs.rest_moments(p.n_theta, p.n_phi)
    og, f_ref, phi_ref = oracle_run(p, phi, n, ut, up, 2000)
    gg, f_gpu, phi_gpu = gpu_run(p, phi, n, ut, up, 2000, precision=32)
    mr, mg = og.moments(), moments_np(gg.moments())
    errs = dict(f=rel_linf(f_gpu, f_ref), phi=rel_linf(phi_gpu, phi_ref),
                n=rel_linf(mg["n"], mr["n"]), ut=rel_linf(mg["u_theta"], mr["u_theta"]),
                up=rel_linf(mg["u_phi"], mr["u_phi"]))
    mo = og.invariants()[0]
    mgpu = gg.invariants()[0]
    errs["mass"] = abs(mgpu - mo) / mo
    print("fp32 vs fp64 oracle", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    bars = dict(f=1.5e-3, phi=1e-3, n=1.5e-3, ut=3e-2, up=3e-2, mass=3e-4)
    for k, v in errs.items():
        assert v <= bars[k], (k, v)


def test_drop_workload_fp32_dense_fluid(torch_cuda):
    """The drop workload at density 20 (the density of the paper's phase-separation runs).
    FP32 grids store deviations from the rest equilibrium of the state's own mean density, so
    the bars of unit density hold: against the FP64 oracle after 2000 steps, and for the mass
    over 20,000 steps (storing deviations from unit density, the mass drifted by 1.8e-2 over
    10^6 steps at this density)."""
    p = inputs.drop_workload()
    phi = inputs.drop_workload_phi(p, seed=1)
    n, ut, up = inputs.rest_moments(p.n_theta, p.n_phi, n0=20.0)
    og, f_ref, phi_ref = oracle_run(p, phi, n, ut, up, 2000)
    gg, f_gpu, phi_gpu = gpu_run(p, phi, n, ut, up, 2000, precision=32)
    mr, mg = og.moments(), moments_np(gg.moments())
    errs = dict(f=rel_linf(f_gpu, f_ref), phi=rel_linf(phi_gpu, phi_ref),
                n=rel_linf(mg["n"], mr["n"]), ut=rel_linf(mg["u_theta"], mr["u_theta"]),
                up=rel_linf(mg["u_phi"], mr["u_phi"]))
    m_exact = 20.0 * 4 * math.pi ** 2 * p.r * p.R
    errs["mass"] = abs(gg.invariants()[0] - m_exact) / m_exact
    gg.step(18000)
    errs["mass_20000"] = abs(gg.invariants()[0] - m_exact) / m_exact
    print("fp32 at density 20 vs fp64 oracle", {k: f"{v:.2e}" for k, v in errs.items()},
          flush=True)
    bars = dict(f=1.5e-3, phi=1e-3, n=1.5e-3, ut=3e-2, up=3e-2, mass=3e-4, mass_20000=1e-5)
    for k, v in errs.items():
        assert v <= bars[k], (k, v)


def test_checkpoint_resume_is_bitwise(torch_cuda):
    p = inputs.TorusParams(1.0, 2.5, 20, 70, 0.5, 2e-3, 0.05, 0.3, 2e-4)
    phi, n, ut, up = inputs.random_state(p, seed=5)
    from paper_1904_10070_amd import TorusGrid
    a = TorusGrid(p, precision=64)
    a.set_state(phi, n, ut, up)
    a.step(10)
    f_mid, phi_mid = (x.clone() for x in a.get_state())
    a.step(10)
    fa, pa = a.get_state()
    b = TorusGrid(p, precision=64)
    b.set_state(phi_mid, f=f_mid)
    b.step(10)
    fb, pb = b.get_state()
    torch_cuda.cuda.synchronize()
    assert torch_cuda.equal(fa, fb) and torch_cuda.equal(pa, pb)


def test_invariants_reproducible_and_nonfinite(torch_cuda):
    p = inputs.TorusParams(1.0, 2.5, 40, 100, 0.5, 2e-3, 0.05, 0.3, 2e-4)
    phi, n, ut, up = inputs.random_state(p, seed=9)
    from paper_1904_10070_amd import TorusGrid
    g = TorusGrid(p, precision=64)
    g.set_state(phi, n, ut, up)
    g.step(3)
    a, b = g.invariants(), g.invariants()
    assert a == b and a[2] == 0
    og, _, _ = oracle_run(p, phi, n, ut, up, 3)
    mo, so, _ = og.invariants()
    assert abs(a[0] - mo) <= 1e-13 * mo and abs(a[1] - so) <= 1e-13 * mo
    # a NaN injected from the host is counted
    bad = phi.copy()
    bad[7, 13] = np.nan
    g.set_state(bad, n, ut, up)
    m, s, cnt = g.invariants()
    assert cnt >= 1


def test_spinodal_full_size_fp64_and_fp32(torch_cuda):
    """512 x 1280, the launch configuration the benchmark times: 2 steps in FP64 against the
    oracle at 1e-12, and in FP32 within the single-precision rounding of 2 steps."""
    p = inputs.spinodal_workload(0.6)
    phi = inputs.spinodal_phi(p, seed=7)
    n, ut, up = inputs.rest_moments(p.n_theta, p.n_phi)
    og, f_ref, phi_ref = oracle_run(p, phi, n, ut, up, 2)
    _, f64, p64 = gpu_run(p, phi, n, ut, up, 2, precision=64)
    assert rel_linf(f64, f_ref) <= FP64_TOL and rel_linf(p64, phi_ref) <= FP64_TOL
    _, f32, p32 = gpu_run(p, phi, n, ut, up, 2, precision=32)
    e32f, e32p = rel_linf(f32, f_ref), rel_linf(p32, phi_ref)
    print(f"512x1280 fp32 after 2 steps: f {e32f:.2e} phi {e32p:.2e}", flush=True)
    assert e32f <= 1e-5 and e32p <= 1e-5


@pytest.mark.timeout(300)
def test_roofline_size_streaming_fp64_and_fp32(torch_cuda):
    """2048 x 5120, whose state copies (2.1 GB in FP32, 4.3 GB in FP64) are far beyond the
    last-level cache, so the stage kernel streams its outputs and the y^n loads past the
    caches: 2 steps against the oracle, FP64 at 1e-12 and FP32 within single-precision
    rounding (the launch configuration the benchmark times for this grid)."""
    p = inputs.roofline_workload()
    phi = inputs.spinodal_phi(p, seed=7)
    n, ut, up = inputs.rest_moments(p.n_theta, p.n_phi)
    og, f_ref, phi_ref = oracle_run(p, phi, n, ut, up, 2)
    del og
    g, f64, p64 = gpu_run(p, phi, n, ut, up, 2, precision=64)
    g.close()
    e64f, e64p = rel_linf(f64, f_ref), rel_linf(p64, phi_ref)
    del f64, p64
    g, f32, p32 = gpu_run(p, phi, n, ut, up, 2, precision=32)
    g.close()
    e32f, e32p = rel_linf(f32, f_ref), rel_linf(p32, phi_ref)
    print(f"2048x5120 after 2 steps: fp64 f {e64f:.2e} phi {e64p:.2e}; "
          f"fp32 f {e32f:.2e} phi {e32p:.2e}", flush=True)
    assert e64f <= FP64_TOL and e64p <= FP64_TOL
    assert e32f <= 1e-5 and e32p <= 1e-5


@pytest.mark.parametrize("precision", [64, 32])
def test_graph_replay_matches_plain_launches_bitwise(torch_cuda, precision):
    """tlb_step_n replays a prebuilt graph of 32 steps; with TLB_NO_GRAPH it launches each
    kernel.  Several replays, with eager work and synchronisation between them, must give
    bit-identical states."""
    from paper_1904_10070_amd import TorusGrid, NO_GRAPH
    p = inputs.TorusParams(1.0, 2.5, 40, 96, 0.5, 2e-3, 0.05, 0.3, 2e-4)
    phi, n, ut, up = inputs.random_state(p, seed=17)
    a = TorusGrid(p, precision=precision)
    b = TorusGrid(p.with_(flags=NO_GRAPH), precision=precision)
    for g in (a, b):
        g.set_state(phi, n, ut, up)
    for call in range(5):
        a.step(64 + call)       # 2 graph replays + call plain steps
        b.step(64 + call)
        a.moments()
        torch_cuda.cuda.synchronize()
        fa, pa = a.get_state()
        fb, pb = b.get_state()
        assert torch_cuda.equal(fa, fb) and torch_cuda.equal(pa, pb), call


@pytest.mark.parametrize("flags", [0, 4])
def test_fp32_state_does_not_depend_on_how_steps_are_split(torch_cuda, flags):
    """FP32 grids keep the order parameter as a base plus a deviation and fold the deviation
    into the base after every 32nd step since set_state.  That schedule counts steps, not
    calls: 100 steps in one call and the same 100 steps in calls of 7, 45 and 48 (graph
    replays, flags 0, or launch by launch, flags 4 = TLB_NO_GRAPH) give the same bits."""
    from paper_1904_10070_amd import TorusGrid
    p = inputs.TorusParams(1.0, 2.5, 40, 96, 0.5, 2e-3, 0.05, 0.3, 2e-4)
    state = inputs.random_state(p, seed=23)
    a = TorusGrid(p, precision=32)
    b = TorusGrid(p.with_(flags=flags), precision=32)
    for g in (a, b):
        g.set_state(*state)
    a.step(100)
    for k in (7, 45, 48):
        b.step(k)
    fa, pa = a.get_state()
    fb, pb = b.get_state()
    torch_cuda.cuda.synchronize()
    assert torch_cuda.equal(fa, fb) and torch_cuda.equal(pa, pb)


@pytest.mark.parametrize("shape,flags", [((64, 160), 8), ((37, 150), 8), ((9, 70), 8 | 1),
                                         ((24, 96), 8 | 2)])
def test_weno5_variant_fp64(torch_cuda, shape, flags):
    """The WENO-5 advection variant (flag 8) against the oracle's, alone and with the flat and
    no-CH-advection flags, on a drop and on random states (ragged tiles)."""
    nt, np_ = shape
    if shape == (64, 160):
        p = inputs.drop_workload().with_(flags=flags)
        phi = inputs.drop_workload_phi(p, seed=1)
        n, ut, up = inputs.rest_moments(nt, np_)
        steps = 400
    else:
        p = inputs.TorusParams(1.0, 2.5, nt, np_, 0.5, 2e-3, 0.05, 0.3, 2e-4, flags)
        phi, n, ut, up = inputs.random_state(p, seed=nt + np_)
        steps = 25
    compare_fp64(p, phi, n, ut, up, steps, flags_note=f"WENO flags={flags}")


def test_weno5_variant_fp32_tolerance(torch_cuda):
    p = inputs.drop_workload().with_(flags=8)
    phi = inputs.drop_workload_phi(p, seed=1)
    n, ut, up = inputs.rest_moments(p.n_theta, p.n_phi)
    og, f_ref, phi_ref = oracle_run(p, phi, n, ut, up, 2000)
    gg, f_gpu, phi_gpu = gpu_run(p, phi, n, ut, up, 2000, precision=32)
    ef, ep = rel_linf(f_gpu, f_ref), rel_linf(phi_gpu, phi_ref)
    print(f"WENO fp32 vs fp64 oracle: f {ef:.2e} phi {ep:.2e}", flush=True)
    assert ef <= 1.5e-3 and ep <= 1e-3


def test_uneven_mixture_64x160_fp64_2000_steps(torch_cuda):
    """An uneven mixture (section IV: mean order parameter -0.3) on the 64 x 160 torus with the
    drop workload's parameters: phi = -0.3 + U(-0.1, 0.1) (eq. phirand with a shifted mean),
    2000 steps, FP64 against the oracle at 1e-12; both keep the mean of phi (the J-weighted sum
    over the area) at -0.3."""
    p = inputs.drop_workload()
    phi = inputs.spinodal_phi(p, seed=3, mean=-0.3)
    n, ut, up = inputs.rest_moments(p.n_theta, p.n_phi)
    og, gg = compare_fp64(p, phi, n, ut, up, 2000, flags_note="mean phi -0.3")
    area = 4 * math.pi ** 2 * p.r * p.R
    for g in (og, gg):
        m, s, bad = g.invariants()
        assert bad == 0
        assert abs(s / area + 0.3) <= 2e-3    # the initial noise has a sample mean near 0


def test_uneven_mixture_full_size_fp64_and_fp32(torch_cuda):
    """The 512 x 1280 spinodal workload with mean order parameter -0.3: 2 steps, FP64 against
    the oracle at 1e-12 (f, phi, moments and mu) and FP32 within the rounding of 2 steps."""
    p = inputs.spinodal_workload(0.6)
    phi = inputs.spinodal_phi(p, seed=7, mean=-0.3)
    n, ut, up = inputs.rest_moments(p.n_theta, p.n_phi)
    og, gg = compare_fp64(p, phi, n, ut, up, 2, flags_note="mean phi -0.3")
    f_ref, phi_ref = og.get_state()
    gg.close()
    g32, f32, p32 = gpu_run(p, phi, n, ut, up, 2, precision=32)
    e32f, e32p = rel_linf(f32, f_ref), rel_linf(p32, phi_ref)
    print(f"512x1280 mean -0.3 fp32 after 2 steps: f {e32f:.2e} phi {e32p:.2e}", flush=True)
    assert e32f <= 1e-5 and e32p <= 1e-5


@pytest.mark.parametrize("shape,flags", [((64, 160), 32), ((37, 150), 32), ((9, 70), 32 | 1),
                                         ((24, 96), 32 | 2), ((6, 1), 32), ((4, 64), 32 | 4)])
def test_ch4_variant_fp64(torch_cuda, shape, flags):
    """The fourth-order Cahn-Hilliard variant (flag 32: prepass of mu and the advection
    fluxes, fourth-order operators in the stage kernel) against the oracle's, alone and with
    the flat, no-CH-advection and no-graph flags, on a drop and on random states (ragged tiles,
    grids narrower than the stencils)."""
    nt, np_ = shape
    if shape == (64, 160):
        p = inputs.drop_workload().with_(flags=flags)
        phi = inputs.drop_workload_phi(p, seed=1)
        n, ut, up = inputs.rest_moments(nt, np_)
        steps = 400
    else:
        p = inputs.TorusParams(1.0, 2.5, nt, np_, 0.5, 2e-3, 0.05, 0.3, 2e-4, flags)
        phi, n, ut, up = inputs.random_state(p, seed=nt + 3 * np_)
        steps = 40
    compare_fp64(p, phi, n, ut, up, steps, flags_note=f"CH4 flags={flags}")


def test_ch4_variant_fp32_tolerance(torch_cuda):
    """The drop workload with the fourth-order variant in FP32 against the FP64 oracle after
    2000 steps, within the FP32 bars of the second-order scheme."""
    p = inputs.drop_workload().with_(flags=32)
    phi = inputs.drop_workload_phi(p, seed=1)
    n, ut, up = inputs.rest_moments(p.n_theta, p.n_phi)
    og, f_ref, phi_ref = oracle_run(p, phi, n, ut, up, 2000)
    gg, f_gpu, phi_gpu = gpu_run(p, phi, n, ut, up, 2000, precision=32)
    ef, ep = rel_linf(f_gpu, f_ref), rel_linf(phi_gpu, phi_ref)
    mr, mg = og.moments(), moments_np(gg.moments())
    en = rel_linf(mg["n"], mr["n"])
    print(f"CH4 fp32 vs fp64 oracle: f {ef:.2e} phi {ep:.2e} n {en:.2e}", flush=True)
    assert ef <= 1.5e-3 and ep <= 1e-3 and en <= 1.5e-3


def test_ch4_graph_replay_matches_plain_launches_bitwise(torch_cuda):
    """Two kernels per stage in the replayed graphs (prepass and stage kernel): graph replays
    and plain launches give the same bits over several calls."""
    from paper_1904_10070_amd import TorusGrid, NO_GRAPH
    p = inputs.TorusParams(1.0, 2.5, 40, 96, 0.5, 2e-3, 0.05, 0.3, 2e-4, 32)
    phi, n, ut, up = inputs.random_state(p, seed=27)
    a = TorusGrid(p, precision=64)
    b = TorusGrid(p.with_(flags=32 | NO_GRAPH), precision=64)
    for g in (a, b):
        g.set_state(phi, n, ut, up)
    for call in range(3):
        a.step(40 + call)
        b.step(40 + call)
        torch_cuda.cuda.synchronize()
        fa, pa = a.get_state()
        fb, pb = b.get_state()
        assert torch_cuda.equal(fa, fb) and torch_cuda.equal(pa, pb), call
