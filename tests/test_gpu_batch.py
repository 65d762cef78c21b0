"""Tile-height independence, the autotuner, and ensembles of tori in one fused launch.

Every node runs the same arithmetic whatever the tile height or the batching, so results must
be bit-identical: stepping a grid with 4-, 8- or 16-row tiles, after autotuning, or as part of a
batch of tori of different sizes, aspect ratios and time steps gives the same state as
stepping it alone (which the parity tests tie to the oracle).  The bit-exact tile-seam check
also catches halo races between the LDS tiles.
"""

import numpy as np
import pytest

from paper_1904_10070_amd import inputs

pytestmark = pytest.mark.gpu


def make(p, precision, seed, rows=None):
    from paper_1904_10070_amd import TorusGrid
    g = TorusGrid(p, precision=precision)
    if rows:
        g.set_tile_rows(rows)
    g.set_state(*inputs.random_state(p, seed=seed))
    return g


@pytest.mark.parametrize("precision", [64, 32])
def test_tile_height_does_not_change_results(torch_cuda, precision):
    p = inputs.TorusParams(1.0, 2.5, 52, 200, 0.5, 2e-3, 0.05, 0.3, 2e-4)
    states = []
    for rows in (4, 8, 16):
        g = make(p, precision, seed=3, rows=rows)
        g.step(40)
        states.append(g.get_state())
    for f, ph in states[1:]:
        assert torch_cuda.equal(f, states[0][0]) and torch_cuda.equal(ph, states[0][1])


def test_autotune_picks_a_height_and_keeps_results(torch_cuda):
    p = inputs.spinodal_workload(0.6)
    a = make(p, 32, seed=7)
    b = make(p, 32, seed=7)
    rows = a.autotune()
    assert rows in (4, 8, 16)
    a.step(40)
    b.step(40)
    fa, pa = a.get_state()
    fb, pb = b.get_state()
    assert torch_cuda.equal(fa, fb) and torch_cuda.equal(pa, pb)


def ensemble(n, seed, precision):
    """n small tori: R/r in [1.5, 5], grids from 16 x 40 to 64 x 200 (some ragged), own dt."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        R = float(rng.uniform(1.5, 5.0))
        nt = int(rng.choice([16, 24, 40, 64]))
        np_ = int(rng.choice([40, 64, 96, 130, 200]))
        dt = float(rng.uniform(1e-4, 3e-4))
        out.append(inputs.TorusParams(1.0, R, nt, np_, 0.5, 2e-3, 0.05, 0.3, dt))
    return out


@pytest.mark.parametrize("precision", [64, 32])
def test_batch_equals_grids_stepped_alone(torch_cuda, precision):
    from paper_1904_10070_amd import TorusBatch
    params = ensemble(7, seed=5, precision=precision)
    alone = [make(p, precision, seed=100 + i) for i, p in enumerate(params)]
    batched = [make(p, precision, seed=100 + i) for i, p in enumerate(params)]
    batch = TorusBatch(batched)
    for g in alone:
        g.step(70)
    batch.step(70)              # two graph replays of 32 steps + 6 single launches
    torch_cuda.cuda.synchronize()
    for g, h in zip(alone, batched):
        fa, pa = g.get_state()
        fb, pb = h.get_state()
        assert torch_cuda.equal(fa, fb) and torch_cuda.equal(pa, pb)
    rows = batch.autotune()
    assert rows in (4, 8, 16)
    for g in alone:
        g.step(33)
    batch.step(33)
    for g, h in zip(alone, batched):
        assert torch_cuda.equal(g.get_state()[0], h.get_state()[0])
    # grids that were stepped alone before joining a batch: FP32 grids fold the order
    # parameter's deviation into its base on their own step counts, inside the batch too
    alone[0].step(5)
    batched[0].step(5)
    alone[1].step(19)
    batched[1].step(19)
    for g in alone:
        g.step(40)
    batch.step(40)
    torch_cuda.cuda.synchronize()
    for g, h in zip(alone, batched):
        fa, pa = g.get_state()
        fb, pb = h.get_state()
        assert torch_cuda.equal(fa, fb) and torch_cuda.equal(pa, pb)


def test_new_reference_density_reaches_graphs_and_batches(torch_cuda):
    """FP32 grids store deviations from the rest equilibrium of a reference density taken from
    the loaded state.  Reloading a grid with a state of another mean density (here 20 after 1)
    changes it after a graph of its steps or a batch holding it was built: both must pick up
    the new stage arguments, so the grid ends bit for bit where a fresh grid ends."""
    from paper_1904_10070_amd import TorusBatch, TorusGrid
    p = inputs.TorusParams(1.0, 2.5, 40, 100, 0.5, 2e-3, 0.05, 0.3, 2e-4)
    phi, n, ut, up = inputs.random_state(p, seed=21)
    dense = (phi, 20.0 * n, ut, up)

    def fresh(steps):
        g = TorusGrid(p, precision=32)
        g.set_state(*dense)
        g.step(steps)
        return g.get_state()

    single = make(p, 32, seed=22)
    single.step(64)                       # builds and replays the step graph
    single.set_state(*dense)
    single.step(40)
    other = make(p, 32, seed=23)
    member = make(p, 32, seed=24)
    batch = TorusBatch([other, member])
    batch.step(40)                        # builds the table and the batch graph
    member.set_state(*dense)
    batch.step(40)
    ref = fresh(40)
    torch_cuda.cuda.synchronize()
    for g in (single, member):
        f, ph = g.get_state()
        assert torch_cuda.equal(f, ref[0]) and torch_cuda.equal(ph, ref[1])


def test_weno_grids_keep_their_tile_and_stay_out_of_batches(torch_cuda):
    from paper_1904_10070_amd import TorusGrid, TorusBatch, TlbError, WENO5
    p = inputs.TorusParams(1.0, 2.5, 16, 64, 0.5, 2e-3, 0.05, 0.3, 2e-4, WENO5)
    g = TorusGrid(p, precision=32)
    assert g.autotune() == 8
    with pytest.raises(TlbError):
        g.set_tile_rows(4)
    g.set_tile_rows(8)
    with pytest.raises(TlbError):
        TorusBatch([g])


@pytest.mark.timeout(300)
def test_benchmark_ensemble_matches_grids_alone(torch_cuda):
    """The ensemble the benchmark times: 64 tori of 128..512 x 256..1024 nodes (15.2 M in all,
    FP32, seeded spinodal states, autotuned tile height).  After 40 steps (one graph replay of
    32 steps and 8 single launches) every torus is bit for bit where it is when stepped alone."""
    from paper_1904_10070_amd import TorusBatch, TorusGrid
    params = inputs.ensemble_workload()

    def grids():
        out = []
        for i, p in enumerate(params):
            g = TorusGrid(p, precision=32)
            g.set_state(inputs.spinodal_phi(p, seed=1000 + i),
                        *inputs.rest_moments(p.n_theta, p.n_phi))
            out.append(g)
        return out

    batched = grids()
    batch = TorusBatch(batched)
    rows = batch.autotune()
    batch.step(40)
    alone = grids()
    for g in alone:
        g.step(40)
    torch_cuda.cuda.synchronize()
    print(f"64 tori, {sum(p.n_theta * p.n_phi for p in params)} nodes, tile rows {rows}",
          flush=True)
    for i, (g, h) in enumerate(zip(alone, batched)):
        fa, pa = g.get_state()
        fb, pb = h.get_state()
        assert torch_cuda.equal(fa, fb) and torch_cuda.equal(pa, pb), i
    batch.close()
    for g in alone + batched:
        g.close()


def mixed_ensemble(n, seed):
    """n tori with different minor radii (0.6 .. 1.2), aspect ratios R/r in [1.5, 5], grid sizes
    (some ragged: n_phi not a multiple of 64, n_theta not of the tile height) and time steps."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        r = float(rng.uniform(0.6, 1.2))
        R = r * float(rng.uniform(1.5, 5.0))
        nt = int(rng.choice([12, 24, 37, 64]))
        np_ = int(rng.choice([40, 64, 96, 130, 200]))
        dt = float(rng.uniform(1e-4, 2e-4))
        out.append(inputs.TorusParams(r, R, nt, np_, 0.5, 2e-3, 0.05, 0.3, dt))
    return out


def test_batch_matches_oracle_fp64(torch_cuda):
    """Each torus of a mixed ensemble stepped 70 times by tlb_batch_step_n (two replays of the
    32-step batch graph and six single launches) against the CPU oracle stepping it alone:
    f, phi, n and mu within 1e-12 relative, u within 1e-12 of the size of the terms it sums
    (as in the single-grid parity tests)."""
    from paper_1904_10070_amd import TorusBatch, TorusGrid
    from tests.helpers import oracle_run, rel_linf, velocity_scale
    params = mixed_ensemble(6, seed=31)
    states = [inputs.random_state(p, seed=300 + i) for i, p in enumerate(params)]
    grids = []
    for p, st in zip(params, states):
        g = TorusGrid(p, precision=64)
        g.set_state(*st)
        grids.append(g)
    batch = TorusBatch(grids)
    batch.step(70)
    torch_cuda.cuda.synchronize()
    for i, (p, st, g) in enumerate(zip(params, states, grids)):
        og, f_ref, phi_ref = oracle_run(p, *st, 70)
        f, ph = (x.cpu().numpy() for x in g.get_state())
        mg = {k: v.cpu().numpy() for k, v in g.moments().items()}
        mr = og.moments()
        errs = {"f": rel_linf(f, f_ref), "phi": rel_linf(ph, phi_ref)}
        for k in ("n", "mu"):
            errs[k] = rel_linf(mg[k], mr[k])
        for axis, k in enumerate(("u_theta", "u_phi")):
            errs[k] = float(np.abs(mg[k] - mr[k]).max()) / velocity_scale(f_ref, mr["n"], axis)
        print(f"torus {i}: r={p.r:.3f} R={p.R:.3f} {p.n_theta}x{p.n_phi} dt={p.dt:.2e}",
              {k: f"{v:.1e}" for k, v in errs.items()}, flush=True)
        for k, v in errs.items():
            assert v <= 1e-12, (i, k, v)


@pytest.mark.timeout(300)
def test_benchmark_ensemble_fp32_matches_oracle(torch_cuda):
    """The benchmark's 64-torus FP32 ensemble (3.1 GB of state copies: the streaming form of the
    batched launch) after 2 batched steps, each torus against the FP64 oracle: within the FP32
    rounding of two steps (the bar of the single-grid full-size test, 1e-5 relative)."""
    from paper_1904_10070_amd import TorusBatch, TorusGrid
    from tests.helpers import oracle_run, rel_linf
    params = inputs.ensemble_workload()
    grids, phis = [], []
    for i, p in enumerate(params):
        g = TorusGrid(p, precision=32)
        phis.append(inputs.spinodal_phi(p, seed=1000 + i))
        g.set_state(phis[-1], *inputs.rest_moments(p.n_theta, p.n_phi))
        grids.append(g)
    batch = TorusBatch(grids)
    batch.autotune()
    batch.step(2)
    torch_cuda.cuda.synchronize()
    worst = 0.0
    for i, (p, g) in enumerate(zip(params, grids)):
        _, f_ref, phi_ref = oracle_run(p, phis[i], *inputs.rest_moments(p.n_theta, p.n_phi), 2)
        f, ph = (x.double().cpu().numpy() for x in g.get_state())
        ef, ep = rel_linf(f, f_ref), rel_linf(ph, phi_ref)
        worst = max(worst, ef, ep)
        assert ef <= 1e-5 and ep <= 1e-5, (i, ef, ep)
        g.close()
    print(f"64-torus ensemble, 2 steps FP32 vs FP64 oracle: worst rel Linf {worst:.2e}",
          flush=True)
