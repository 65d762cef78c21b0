"""The failure paths of the step loop, on the GPU through the C interface: the non-finite
check of tlb_step_n (check_every) and the stability guard (TLB_STRICT_DT, tlb_stable_dt).
Every kernel of these runs exits normally: a NaN or an unstable time step only makes values
non-finite, which the checks then report."""
import math

import numpy as np
import pytest

from paper_1904_10070_amd import inputs

pytestmark = pytest.mark.gpu


def drop_grid(precision, check_every=0, dt=None, flags=0):
    from paper_1904_10070_amd import TorusGrid
    p = inputs.drop_workload()
    if dt is not None:
        p = p.with_(dt=dt)
    p = p.with_(flags=flags)
    g = TorusGrid(p, precision=precision, check_every=check_every)
    g.set_state(inputs.drop_workload_phi(p, seed=1), *inputs.rest_moments(p.n_theta, p.n_phi))
    return p, g


@pytest.mark.parametrize("precision", [64, 32])
def test_checked_run_is_bitwise_the_unchecked_one(torch_cuda, precision):
    """Checks read the state only: 100 steps checked every 30 (and at the end) give the same
    bits as 100 unchecked steps, and report nothing."""
    _, a = drop_grid(precision, check_every=30)
    _, b = drop_grid(precision)
    a.step(100)
    b.step(100)
    fa, pa = a.get_state()
    fb, pb = b.get_state()
    torch_cuda.cuda.synchronize()
    assert torch_cuda.equal(fa, fb) and torch_cuda.equal(pa, pb)


@pytest.mark.parametrize("precision", [64, 32])
def test_nan_injected_mid_run_is_reported(torch_cuda, precision):
    from paper_1904_10070_amd import TlbError
    from paper_1904_10070_amd.binding import TLB_ENONFINITE
    _, g = drop_grid(precision, check_every=16)
    g.step(40)                                    # clean: no error
    with torch_cuda.cuda.stream(g.stream):
        g.f[0][5, 20, 77] = float("nan")          # one population of one node
    with pytest.raises(TlbError) as e:
        g.step(40)
    assert e.value.code == TLB_ENONFINITE
    assert g.invariants()[2] > 0                  # the state is non-finite, as reported


def test_unstable_time_step_is_reported_by_the_checks(torch_cuda):
    """dt four times the bound of tlb_stable_dt: the Cahn-Hilliard part blows up; without the
    strict flag creation succeeds and the checked run reports non-finite values."""
    from paper_1904_10070_amd import TlbError, stable_dt
    from paper_1904_10070_amd.binding import TLB_ENONFINITE
    p = inputs.drop_workload()
    bound = stable_dt(p)
    assert p.dt < bound                           # the workload itself is stable
    _, g = drop_grid(64, check_every=100, dt=4.0 * bound)
    with pytest.raises(TlbError) as e:
        g.step(400)
    assert e.value.code == TLB_ENONFINITE


def test_strict_flag_refuses_the_unstable_time_step(torch_cuda):
    from paper_1904_10070_amd import TlbError, TorusGrid, STRICT_DT, stable_dt
    from paper_1904_10070_amd.binding import TLB_EUNSTABLE
    p = inputs.drop_workload()
    bound = stable_dt(p)
    with pytest.raises(TlbError) as e:
        TorusGrid(p.with_(dt=4.0 * bound, flags=STRICT_DT), precision=64)
    assert e.value.code == TLB_EUNSTABLE
    g = TorusGrid(p.with_(flags=STRICT_DT), precision=64, check_every=500)   # 5e-4 < bound
    g.set_state(inputs.drop_workload_phi(p, seed=1), *inputs.rest_moments(p.n_theta, p.n_phi))
    g.step(1000)
    m, s, bad = g.invariants()
    assert bad == 0 and math.isfinite(m)
