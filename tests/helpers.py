"""Shared test helpers: relative error norms and oracle/GPU drivers on the same inputs."""
import numpy as np


def rel_linf(a, b):
    """max |a - b| / max |b| (0 if both vanish)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    num = np.abs(a - b).max()
    return float(num / den) if den > 0 else float(num)


def oracle_run(p, phi, n, ut, up, steps, bits=64, f=None):
    from oracle import ref
    g = ref.RefGrid(**p.as_dict(), bits=bits)
    if f is None:
        g.set_state(phi, n, ut, up)
    else:
        g.set_state(phi, f=f)
    if steps:
        g.step(steps)
    f_out, phi_out = g.get_state()
    return g, f_out, phi_out


def gpu_run(p, phi, n, ut, up, steps, precision=64, f=None):
    from paper_1904_10070_amd import TorusGrid
    g = TorusGrid(p, precision=precision)
    if f is None:
        g.set_state(phi, n, ut, up)
    else:
        g.set_state(phi, f=f)
    if steps:
        g.step(steps)
    f_out, phi_out = g.get_state()
    return g, f_out.double().cpu().numpy(), phi_out.double().cpu().numpy()


def velocity_scale(f, n, axis):
    """max over nodes of sum_k |f_k| |v_k| / n along one velocity axis (0: theta, 1: phi): the
    size of the terms whose sum is n u, against which the rounding of u is measured."""
    from oracle import ref
    v = np.asarray(ref.velocity_set()[0], dtype=np.float64)
    i, j = np.divmod(np.arange(16), 4)
    w = np.abs(v[i] if axis == 0 else v[j])
    return float(((np.abs(f) * w[:, None, None]).sum(axis=0) / n).max())
