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
