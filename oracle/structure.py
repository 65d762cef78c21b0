"""Structure-factor length of an order-parameter field on the torus grid (numpy, FP64).

TEST INFRASTRUCTURE ONLY: the CPU reference of tlb_structure_length.  Only tests, the smoke
check and the benchmark's CPU-baseline leg may import it.

Coarsening length from the 2-D power spectrum of phi - <phi> on the (theta, phi) node grid, in
the coordinate-space approximation of the torus: mode (m, m') has wavenumbers
k_theta = m / r and k_phi = m' / R (m, m' the signed mode numbers), and

    S(m, m') = |sum_{q,s} (phi_qs - <phi>) exp(-2 pi i (m q / N_theta + m' s / N_phi))|^2,
    L_S = 2 pi sum S / sum |k| S        (the zero mode carries no power).

The paper measures coarsening by L_d = A_total / L_I (section IV, eq. cart_scaling_L0); L_S is
the structure-factor length of the spinodal workload's specification, computed beside it.
"""
import math

import numpy as np


def signed_modes(n):
    """Mode numbers 0, 1, ..., -1 in FFT order (the Nyquist mode of an even n counts as -n/2)."""
    return np.fft.fftfreq(n, d=1.0 / n)


def structure_length(phi, r, R):
    """(L_S, sum S, sum |k| S) of a field phi[n_theta, n_phi]."""
    phi = np.asarray(phi, dtype=np.float64)
    S = np.abs(np.fft.fft2(phi - phi.mean())) ** 2
    kt = signed_modes(phi.shape[0]) / r
    kp = signed_modes(phi.shape[1]) / R
    k = np.sqrt(kt[:, None] ** 2 + kp[None, :] ** 2)
    s0 = float(S.sum())
    s1 = float((k * S).sum())
    return (2.0 * math.pi * s0 / s1 if s1 > 0 else math.inf), s0, s1
