"""Seeded synthetic inputs: parameter sets and initial fields for the torus workloads.

This module holds no step arithmetic of the method.  It builds the initial order parameter
and the moments (n, u) from which both the GPU library and the CPU oracle set their own
equilibrium populations; both sides receive the very same host arrays.

Initial conditions follow the paper:
  * stripe: tanh profile with the Laplace-pressure offset phi_0 (section III A, eqs.
    stripe_tanh and stripe_phi0);
  * drop: tanh of the 3-D chord distance to the drop centre (section III D, eq. drop_init);
  * spinodal: phi = mean + uniform noise in (-0.1, 0.1) (section IV, eq. phirand);
  * populations at rest: f = f_eq(n0, u = 0) (section IV).

Parameter sets: lengths in units of the minor radius r; k_B T = m = 1 so nu = tau.  The
interface-width rule of the "interface about 3 cells" workloads is
xi_0 = 3 h_max / (2 sqrt 2), h_max = max(r dtheta, 2 pi (R + r) / N_phi), kappa = A xi_0^2
(xi_0 = sqrt(kappa / A), eq. xi_gamma).
"""
import math
from dataclasses import dataclass, asdict, replace

import numpy as np


@dataclass(frozen=True)
class TorusParams:
    r: float
    R: float
    n_theta: int
    n_phi: int
    A: float
    kappa: float
    M: float
    tau: float
    dt: float
    flags: int = 0

    def as_dict(self):
        return asdict(self)

    def with_(self, **kw):
        return replace(self, **kw)

    @property
    def xi0(self):
        return math.sqrt(self.kappa / self.A)

    @property
    def gamma(self):
        return math.sqrt(8.0 * self.kappa * self.A / 9.0)


def xi0_three_cells(r, R, n_theta, n_phi):
    h_max = max(r * 2 * math.pi / n_theta, 2 * math.pi * (R + r) / n_phi)
    return 3.0 * h_max / (2.0 * math.sqrt(2.0))


def params_three_cells(r, R, n_theta, n_phi, A, M, tau, dt, flags=0):
    xi0 = xi0_three_cells(r, R, n_theta, n_phi)
    return TorusParams(r, R, n_theta, n_phi, A, A * xi0 * xi0, M, tau, dt, flags)


# -- the named workloads ------------------------------------------------------------------------

def drop_workload():
    """64 x 160 torus, r = 1, R = 2.5, one drop of radius 0.6 near theta = pi/2; 2000 steps."""
    return params_three_cells(1.0, 2.5, 64, 160, A=0.5, M=0.1, tau=0.8, dt=5e-4)


def stripe_workload(R=2.0, n_theta=256, n_phi=640):
    """Stripe relaxation: r = 1, kappa = 5e-4, A = 0.5, nu = tau = M = 2.5e-3, dt = 5e-4."""
    return TorusParams(1.0, R, n_theta, n_phi, 0.5, 5e-4, 2.5e-3, 2.5e-3, 5e-4)


def spinodal_workload(tau=0.6, n_theta=512, n_phi=1280):
    """Spinodal coarsening: r = 1, R = 2.5, M = 2.5e-3, tau 0.6 or 2.0, dt = 4e-4."""
    return params_three_cells(1.0, 2.5, n_theta, n_phi, A=0.5, M=2.5e-3, tau=tau, dt=4e-4)


def roofline_workload():
    """The spinodal workload on a 2048 x 5120 grid (working set far above the 256 MB MALL)."""
    p = spinodal_workload(0.6, 2048, 5120)
    return p.with_(dt=1e-5)


# -- fields ---------------------------------------------------------------------------------------

def angles(n_theta, n_phi):
    th = np.arange(n_theta) * (2 * np.pi / n_theta)
    ph = np.arange(n_phi) * (2 * np.pi / n_phi)
    return th, ph


def rest_moments(n_theta, n_phi, n0=1.0):
    """(n, u_theta, u_phi) of a fluid at rest with uniform density n0."""
    shape = (n_theta, n_phi)
    return np.full(shape, float(n0)), np.zeros(shape), np.zeros(shape)


def periodic_distance(a, b):
    """Smallest angular distance |a - b| on the circle, in [0, pi]."""
    d = np.mod(a - b, 2 * np.pi)
    return np.minimum(d, 2 * np.pi - d)


def stripe_offset(xi0, R, a, theta_c, dtheta):
    """Laplace-pressure offset phi_0 of eq. stripe_phi0."""
    return (xi0 / (3 * R * math.sqrt(2.0)) * math.cos(theta_c) * math.sin(dtheta / 2) /
            (1 + a * math.cos(theta_c) * math.cos(dtheta / 2)))


def stripe_phi(p, theta_c, dtheta, offset=True, sign=1.0):
    """Stripe of angular width dtheta centred on theta_c (eq. stripe_tanh), phi-independent.

    sign = +1 gives the paper's convention (the stripe is the phi = -1 minority phase);
    sign = -1 is its phi -> -phi image (a phi = +1 band).
    """
    th, _ = angles(p.n_theta, p.n_phi)
    xi0 = p.xi0
    phi0 = stripe_offset(xi0, p.R, p.r / p.R, theta_c, dtheta) if offset else 0.0
    prof = phi0 + np.tanh(p.r / (xi0 * math.sqrt(2.0)) *
                          (periodic_distance(th, theta_c) - dtheta / 2))
    return sign * np.repeat(prof[:, None], p.n_phi, axis=1)


def torus_xyz(r, R, th, ph):
    """Embedding of eq. torus."""
    rho = R + r * np.cos(th)
    return rho * np.cos(ph), rho * np.sin(ph), r * np.sin(th)


def drop_phi(p, theta0, phi0, R0, xi0=None):
    """tanh((d - R0)/(xi0 sqrt 2)), d the 3-D chord distance to the centre (eq. drop_init)."""
    xi0 = p.xi0 if xi0 is None else xi0
    th, ph = angles(p.n_theta, p.n_phi)
    T, P = np.meshgrid(th, ph, indexing="ij")
    x, y, z = torus_xyz(p.r, p.R, T, P)
    xc, yc, zc = torus_xyz(p.r, p.R, theta0, phi0)
    d = np.sqrt((x - xc) ** 2 + (y - yc) ** 2 + (z - zc) ** 2)
    return np.tanh((d - R0) / (xi0 * math.sqrt(2.0)))


def drop_workload_phi(p, seed=1, R0=0.6):
    """Drop of radius R0 centred at (pi/2, 0) with a seeded +/-1 % jitter of each period."""
    rng = np.random.default_rng(seed)
    u1, u2 = rng.uniform(-0.5, 0.5, size=2)
    return drop_phi(p, 0.5 * np.pi + 0.02 * np.pi * u1, 0.02 * np.pi * u2, R0)


def spinodal_phi(p, seed=7, mean=0.0, amp=0.1):
    """phi = mean + i.i.d. uniform noise in (-amp, amp) (eq. phirand)."""
    rng = np.random.default_rng(seed)
    return mean + rng.uniform(-amp, amp, size=(p.n_theta, p.n_phi))


def random_state(p, seed=0, amp_phi=0.5, amp_u=0.05, amp_n=0.05):
    """A smooth-plus-noise moment state for parity tests away from any equilibrium."""
    rng = np.random.default_rng(seed)
    th, ph = angles(p.n_theta, p.n_phi)
    T, P = np.meshgrid(th, ph, indexing="ij")
    phi = amp_phi * np.sin(T + 0.3) * np.cos(2 * P) + 0.1 * rng.uniform(-1, 1, T.shape)
    n = 1.0 + amp_n * rng.uniform(-1, 1, T.shape)
    ut = amp_u * rng.uniform(-1, 1, T.shape)
    up = amp_u * rng.uniform(-1, 1, T.shape)
    return phi, n, ut, up


# -- time step and ensembles -----------------------------------------------------------------------

def stable_dt(p, safety=0.5):
    """A time step below the explicit stability limits of the discrete step: upwind advection
    at CFL 1 over the smallest spacings, BGK relaxation (2.5 tau, the SSP-RK3 real-axis limit)
    and the Cahn-Hilliard operator (biharmonic M kappa S^2 plus M A 2 S with
    S = 4/h_theta^2 + 4/h_phi^2 at the inner equator, against the same 2.51 limit)."""
    v_max = math.sqrt(3.0 + math.sqrt(6.0))
    h_t = p.r * 2 * math.pi / p.n_theta
    h_p = (p.R - p.r) * 2 * math.pi / p.n_phi
    dt_adv = 1.0 / (v_max * (1.0 / h_t + 1.0 / h_p))
    dt_bgk = 2.5 * p.tau
    S = 4.0 / h_t ** 2 + 4.0 / h_p ** 2
    dt_ch = 2.51 / (p.M * p.kappa * S * S + 2.0 * p.M * abs(p.A) * S + 1e-300)
    return safety * min(dt_adv, dt_bgk, dt_ch)


def ensemble_workload(n=64, seed=4):
    """n tori for coarsening statistics: r = 1, R uniform in [1.5, 5], N_theta from
    {128, 192, ..., 512} and N_phi = 2 N_theta (seeded), interface width by the three-cell
    rule, M = 2.5e-3, tau = 0.6, each with half its stability limit as time step."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        R = float(rng.uniform(1.5, 5.0))
        nt = int(rng.choice(np.arange(128, 513, 64)))
        p = params_three_cells(1.0, R, nt, 2 * nt, A=0.5, M=2.5e-3, tau=0.6, dt=1.0)
        out.append(p.with_(dt=stable_dt(p)))
    return out


# -- the learned coarse-step correction -------------------------------------------------------------

CNN_ARCH = ((6, 32), (32, 32), (32, 32), (32, 32), (32, 4))   # (inputs, outputs) per layer


def cnn_init_params(seed, last_gain=0.1):
    """Seeded He-normal initial weights (std sqrt(2 / (9 c_in))), zero biases, the last layer
    scaled by last_gain; flat FP32 vector, layer by layer W[c_out][9][c_in] then b[c_out]."""
    rng = np.random.default_rng(seed)
    parts = []
    for l, (ci, co) in enumerate(CNN_ARCH):
        std = math.sqrt(2.0 / (9 * ci)) * (last_gain if l == len(CNN_ARCH) - 1 else 1.0)
        parts += [rng.normal(0.0, std, size=co * 9 * ci), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


def learn_samples(seed, n, n_theta, n_phi):
    """Seeded synthetic moment samples (phi, n, u_theta, u_phi) and targets, float32
    [n, n_theta, n_phi, 4] each, with the magnitudes of coarse spinodal states and of their
    per-step corrections."""
    rng = np.random.default_rng(seed)
    shape = (n, n_theta, n_phi)
    m = np.stack([rng.uniform(-1, 1, shape), 1 + 0.02 * rng.normal(size=shape),
                  0.01 * rng.normal(size=shape), 0.01 * rng.normal(size=shape)], -1)
    y = rng.normal(size=shape + (4,)) * np.array([1e-3, 1e-6, 1e-5, 1e-5])
    return m.astype(np.float32), y.astype(np.float32)


def random_populations(n_theta, n_phi, seed):
    """Seeded positive populations f[16, n_theta, n_phi] (each in (0.5, 1.5)/16) and
    phi in (-1, 1), float64: states away from any equilibrium for operator tests."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.5, 1.5, size=(16, n_theta, n_phi)) / 16.0
    phi = rng.uniform(-1, 1, size=(n_theta, n_phi))
    return f, phi
