"""Flat, doubly periodic Cartesian binary-fluid lattice Boltzmann solver in numpy (FP64).

TEST INFRASTRUCTURE ONLY.  A second, independently written reference for the flat limit of
the torus model: the same Q = 4 Hermite velocity set, BGK collision, force term through the
Hermite velocity-derivative kernel, and Cahn-Hilliard coupling (section II of the paper), on a
plane with spacings dx (fast axis x, velocity index j) and dy (slow axis y, index i).  Written
with whole-array numpy shifts instead of loops, so it shares no structure with tlb_oracle.c.

The torus step reduces to this one when J = R and G = 0 with dx = R dphi and dy = r dtheta:
that is the flat-limit pin of the torus oracle.

The velocity set and the derivative kernel are rebuilt here from numpy's Gauss-Hermite
quadrature (numpy.polynomial.hermite_e), not from the C oracle.
"""
import math

import numpy as np
from numpy.polynomial import hermite_e as He


def velocity_set():
    """Q = 4 probabilists' Gauss-Hermite nodes/weights and the derivative kernel K[i, m]."""
    Q = 4
    x, wq = He.hermegauss(Q)             # weight exp(-x^2/2), sum wq = sqrt(2 pi)
    w = wq / math.sqrt(2.0 * math.pi)
    # f(v) ~ omega(v) sum_l a_l He_l(v) / l!  with a_l = sum_m f_m He_l(v_m); then
    # d/dv [omega He_l] = -omega He_{l+1}, evaluated at the nodes with the weight w_i.
    K = np.zeros((Q, Q))
    for l in range(Q):
        cl = np.zeros(l + 2); cl[l + 1] = 1.0
        c0 = np.zeros(l + 1); c0[l] = 1.0
        K += -np.outer(w * He.hermeval(x, cl), He.hermeval(x, c0)) / math.factorial(l)
    return x, w, K


class FlatLB:
    def __init__(self, nx, ny, dx, dy, A, kappa, M, tau, dt, ch_advection=True):
        self.nx, self.ny, self.dx, self.dy = nx, ny, dx, dy
        self.A, self.kappa, self.M, self.tau, self.dt = A, kappa, M, tau, dt
        self.ch_advection = ch_advection
        self.v, self.w, self.K = velocity_set()
        # population k = 4 i + j: y-velocity v[i], x-velocity v[j]
        self.vy = np.repeat(self.v, 4)[:, None, None]
        self.vx = np.tile(self.v, 4)[:, None, None]
        self.ww = np.outer(self.w, self.w).reshape(16)[:, None, None]
        self.f = None
        self.phi = None

    # -- shifts: sh(a, o, axis) returns a evaluated at index + o (periodic)
    @staticmethod
    def sh(a, o, axis):
        return np.roll(a, -o, axis=axis)

    def feq(self, n, uy, ux):
        vu = self.vy * uy[None] + self.vx * ux[None]
        u2 = (uy * uy + ux * ux)[None]
        return n[None] * self.ww * (1 + vu + 0.5 * (vu ** 2 - u2) + vu * (vu ** 2 - 3 * u2) / 6)

    def lap(self, a):
        return ((self.sh(a, 1, 1) - 2 * a + self.sh(a, -1, 1)) / self.dx ** 2 +
                (self.sh(a, 1, 0) - 2 * a + self.sh(a, -1, 0)) / self.dy ** 2)

    def ddx_upwind5(self, h, axis, positive):
        """(face_{+1/2} - face_{-1/2}) of the fifth-order upwind reconstruction."""
        c = np.array([2.0, -13.0, 47.0, 27.0, -3.0]) / 60.0
        if positive:
            offs = (-2, -1, 0, 1, 2)
        else:
            offs = (3, 2, 1, 0, -1)
        face_p = sum(ci * self.sh(h, o, axis) for ci, o in zip(c, offs))
        face_m = self.sh(face_p, -1, axis)
        return face_p - face_m

    def rhs(self, f, phi):
        n = f.sum(0)
        uy = (f * self.vy).sum(0) / n
        ux = (f * self.vx).sum(0) / n
        mu = -self.A * phi * (1 - phi ** 2) - self.kappa * self.lap(phi)
        Fy = -phi * (self.sh(mu, 1, 0) - self.sh(mu, -1, 0)) / (2 * self.dy) / n
        Fx = -phi * (self.sh(mu, 1, 1) - self.sh(mu, -1, 1)) / (2 * self.dx) / n
        # Cahn-Hilliard: -div(u phi) + M lap(mu), central differences of the flux
        Lphi = self.M * self.lap(mu)
        if self.ch_advection:
            Py, Px = uy * phi, ux * phi
            Lphi = Lphi - ((self.sh(Py, 1, 0) - self.sh(Py, -1, 0)) / (2 * self.dy) +
                           (self.sh(Px, 1, 1) - self.sh(Px, -1, 1)) / (2 * self.dx))
        # Boltzmann: velocity derivatives through K along each velocity axis
        f4 = f.reshape(4, 4, self.ny, self.nx)            # [i, j, y, x]
        dfdvy = np.einsum("im,mjyx->ijyx", self.K, f4).reshape(16, self.ny, self.nx)
        dfdvx = np.einsum("jm,imyx->ijyx", self.K, f4).reshape(16, self.ny, self.nx)
        Lf = -(Fy[None] * dfdvy + Fx[None] * dfdvx)
        Lf -= (f - self.feq(n, uy, ux)) / self.tau
        for k in range(16):
            vy, vx = self.vy[k, 0, 0], self.vx[k, 0, 0]
            Lf[k] -= vx / self.dx * self.ddx_upwind5(f[k], 1, vx > 0)
            Lf[k] -= vy / self.dy * self.ddx_upwind5(f[k], 0, vy > 0)
        return Lf, Lphi

    def set_state(self, phi, n, uy, ux):
        self.phi = np.array(phi, dtype=np.float64)
        self.f = self.feq(np.asarray(n, float), np.asarray(uy, float), np.asarray(ux, float))

    def step(self, nsteps=1):
        dt = self.dt
        for _ in range(nsteps):
            f0, p0 = self.f, self.phi
            Lf, Lp = self.rhs(f0, p0)
            f1, p1 = f0 + dt * Lf, p0 + dt * Lp
            Lf, Lp = self.rhs(f1, p1)
            f2, p2 = 0.75 * f0 + 0.25 * (f1 + dt * Lf), 0.75 * p0 + 0.25 * (p1 + dt * Lp)
            Lf, Lp = self.rhs(f2, p2)
            self.f = f0 / 3 + 2 / 3 * (f2 + dt * Lf)
            self.phi = p0 / 3 + 2 / 3 * (p2 + dt * Lp)

    def moments(self):
        n = self.f.sum(0)
        return dict(n=n, u_y=(self.f * self.vy).sum(0) / n, u_x=(self.f * self.vx).sum(0) / n,
                    phi=self.phi)
