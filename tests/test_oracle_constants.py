"""Pins of the oracle's velocity space (section II C of the paper) against what the paper and
the mathematics fix: the printed nodes, weights and 4 x 4 derivative kernels, Gauss-Hermite
exactness, and the exactness of the kernel on low-degree Hermite expansions."""
import math
import os

import numpy as np
import pytest

from oracle import ref
from oracle import flat_numpy

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_closed_forms():
    env = {"sqrt": math.sqrt, "s2": math.sqrt(2), "s3": math.sqrt(3), "s6": math.sqrt(6)}
    mats, cur = {}, None
    for line in open(os.path.join(GOLDEN, "kh_closed_forms.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            cur = line.strip("[]")
            mats[cur] = []
            continue
        mats[cur].append([eval(x, {"__builtins__": {}}, env) for x in line.split(";")])
    return {k: np.array(v) for k, v in mats.items()}


@pytest.fixture(scope="module")
def vs():
    return ref.velocity_set()


def test_nodes_are_the_printed_hermite_roots(vs):
    v, w, K, Kt = vs
    printed = np.array([-math.sqrt(3 + math.sqrt(6)), -math.sqrt(3 - math.sqrt(6)),
                        math.sqrt(3 - math.sqrt(6)), math.sqrt(3 + math.sqrt(6))])
    assert np.allclose(v, printed, rtol=0, atol=1e-15)
    he4 = v ** 4 - 6 * v ** 2 + 3  # probabilists' He_4
    assert np.abs(he4).max() < 1e-13


def test_weights_are_the_printed_values(vs):
    v, w, K, Kt = vs
    w14, w23 = (3 - math.sqrt(6)) / 12, (3 + math.sqrt(6)) / 12
    assert np.allclose(w, [w14, w23, w23, w14], rtol=1e-15, atol=0)


def test_gauss_hermite_exact_to_degree_seven(vs):
    v, w, K, Kt = vs
    for s in range(8):
        exact = 0.0 if s % 2 else float(np.prod(np.arange(s - 1, 0, -2))) if s else 1.0
        assert abs((w * v ** s).sum() - exact) < 1e-13, s
    # degree 8 is where a 4-point rule stops being exact: sum w v^8 = 81, not 7!! = 105
    assert abs((w * v ** 8).sum() - 81.0) < 1e-11


def test_kernels_match_printed_closed_forms(vs):
    v, w, K, Kt = vs
    cf = load_closed_forms()
    assert np.abs(K - cf["KH"]).max() < 1e-14
    assert np.abs(Kt - cf["KHT"]).max() < 1e-14


def test_kernel_identities(vs):
    v, w, K, Kt = vs
    # mass conservation of the force terms: every column of K and K~ sums to zero
    assert np.abs(K.sum(axis=0)).max() < 1e-14
    assert np.abs(Kt.sum(axis=0)).max() < 1e-14
    # momentum: sum_i v_i K_im = -1, energy: sum_i v_i^2 K_im = -2 v_m
    assert np.abs(v @ K + 1).max() < 1e-14
    assert np.abs((v ** 2) @ K + 2 * v).max() < 1e-13
    # d(f v)/dv through K~ equals d/dv applied to (v f): K~ = K diag(v)
    assert np.abs(Kt - K * v[None, :]).max() < 1e-14
    # reflection v -> -v: K_{3-i,3-m} = -K_{i,m}
    assert np.abs(K[::-1, ::-1] + K).max() < 1e-14


@pytest.mark.parametrize("coeffs", [(1, 0, 0, 0), (0, 1, 0, 0), (0.3, -0.7, 0.2, 0.1),
                                    (1, 2, -1, 0.5)])
def test_kernel_is_exact_on_cubic_expansions(vs, coeffs):
    """For f(v) = omega(v) P(v) with deg P <= 3 the derivative is omega (P' - v P); its values
    at the nodes (weights in place of omega) must come out of K exactly."""
    v, w, K, Kt = vs
    P = np.polynomial.Polynomial(coeffs)
    f = w * P(v)
    exact = w * (P.deriv()(v) - v * P(v))
    assert np.abs(K @ f - exact).max() < 1e-13


def test_independent_gauss_hermite_construction_agrees(vs):
    """numpy's Gauss-Hermite quadrature (a different algorithm) gives the same set."""
    v, w, K, Kt = vs
    v2, w2, K2 = flat_numpy.velocity_set()
    assert np.abs(v - v2).max() < 1e-14 and np.abs(w - w2).max() < 1e-14
    assert np.abs(K - K2).max() < 1e-13
