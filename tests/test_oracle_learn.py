"""Pins of the learned-correction reference (oracle/cnn_ref.py) against definitions and
identities that do not reuse its code: brute-force loops, scipy's periodic correlation,
torch's bfloat16 conversion, the adjoint identities of a convolution, finite differences of
the exact network, Adam's closed form under a constant gradient, the Fourier symbol of full
weighting and the moment identities of the Hermite equilibrium."""
import math

import numpy as np
import pytest

from oracle import cnn_ref as C
from paper_1904_10070_amd import inputs


def test_architecture_tables_agree():
    assert tuple(inputs.CNN_ARCH) == tuple(C.ARCH)
    assert C.param_count() == 30660 == len(inputs.cnn_init_params(0))


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-3, 500), rng.normal(0, 50, 500)])
    # exact ties between two bfloat16 neighbours, both parities
    x = np.concatenate([x, [1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 0.0]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(C.bf16(x), ref)
    assert C.bf16(np.array([1 + 2.0 ** -8]))[0] == 1.0                 # tie to even
    assert C.bf16(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6     # tie to even (up)


def brute_conv(a, W, b):
    N, H, Wd, Ci = a.shape
    Co = W.shape[0]
    z = np.zeros((N, H, Wd, Co))
    for n in range(N):
        for y in range(H):
            for x in range(Wd):
                for o in range(Co):
                    acc = b[o]
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            t = 3 * (dy + 1) + (dx + 1)
                            for i in range(Ci):
                                acc += W[o, t, i] * a[n, (y + dy) % H, (x + dx) % Wd, i]
                    z[n, y, x, o] = acc
    return z


def test_conv_matches_brute_force_and_scipy():
    from scipy import ndimage
    rng = np.random.default_rng(1)
    a = rng.normal(size=(2, 4, 5, 3))
    W = rng.normal(size=(2, 9, 3))
    b = rng.normal(size=2)
    z = C.conv3x3(a, W, b)
    assert np.allclose(z, brute_conv(a, W, b), rtol=0, atol=1e-12)
    for n in range(2):
        for o in range(2):
            acc = np.full(a.shape[1:3], b[o])
            for i in range(3):
                acc += ndimage.correlate(a[n, :, :, i], W[o, :, i].reshape(3, 3), mode="wrap")
            assert np.allclose(z[n, :, :, o], acc, rtol=0, atol=1e-12)


def test_conv_adjoints():
    """<conv(a; W), e> = <a, conv^T(e; W)> = <W, dW(e, a)> for any a, W, e."""
    rng = np.random.default_rng(2)
    a = rng.normal(size=(3, 6, 7, 4))
    W = rng.normal(size=(5, 9, 4))
    e = rng.normal(size=(3, 6, 7, 5))
    lhs = np.sum(C.conv3x3(a, W) * e)
    mid = np.sum(a * C.conv3x3_transpose(e, W))
    rhs = np.sum(W * C.conv3x3_weight_grad(e, a))
    assert abs(lhs - mid) <= 1e-11 * abs(lhs) and abs(lhs - rhs) <= 1e-11 * abs(lhs)


def small_problem(seed, N=2, H=5, W=6):
    rng = np.random.default_rng(seed)
    m = np.stack([rng.uniform(-1, 1, (N, H, W)), 1 + 0.05 * rng.normal(size=(N, H, W)),
                  0.01 * rng.normal(size=(N, H, W)), 0.01 * rng.normal(size=(N, H, W))], -1)
    y = rng.normal(size=(N, H, W, 4)) * np.array([1e-3, 1e-5, 1e-4, 1e-4])
    geo = dict(r=1.0, R=2.5, shift=[0.0, 1.0, 0.0, 0.0], scale=[1.0, 20.0, 100.0, 100.0],
               out_scale=[1e-3, 1e-5, 1e-4, 1e-4], loss_weight=[2.0, 1.0, 0.5, 0.5])
    params = inputs.cnn_init_params(seed, last_gain=1.0).astype(np.float64)
    params += 0.01 * rng.normal(size=params.shape)        # nonzero biases
    return params, m, y, geo


def test_gradient_matches_finite_differences():
    """Exact network (no rounding): central differences on parameters of every layer."""
    params, m, y, g = small_problem(3)
    L, grad, _ = C.loss_and_grad(params, m, y, g["r"], g["R"], g["shift"], g["scale"],
                                 g["out_scale"], g["loss_weight"], rounding=False)
    sizes = [co * 9 * ci + co for ci, co in C.ARCH]
    starts = np.cumsum([0] + sizes)
    rng = np.random.default_rng(4)
    picks = []
    for l in range(len(C.ARCH)):
        picks += list(rng.integers(starts[l], starts[l + 1] - C.ARCH[l][1], size=6))   # weights
        picks += [starts[l + 1] - 1 - int(rng.integers(C.ARCH[l][1]))]                  # a bias
    h = 1e-6
    for i in picks:
        p1, p2 = params.copy(), params.copy()
        p1[i] += h
        p2[i] -= h
        L1 = C.loss_and_grad(p1, m, y, g["r"], g["R"], g["shift"], g["scale"], g["out_scale"],
                             g["loss_weight"], rounding=False)[0]
        L2 = C.loss_and_grad(p2, m, y, g["r"], g["R"], g["shift"], g["scale"], g["out_scale"],
                             g["loss_weight"], rounding=False)[0]
        fd = (L1 - L2) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * np.abs(grad).max() + 1e-5 * abs(grad[i]), (i, fd, grad[i])


def test_rounded_gradient_close_to_exact():
    """The bfloat16 policy perturbs the gradient by about the bfloat16 precision."""
    params, m, y, g = small_problem(5)
    args = (g["r"], g["R"], g["shift"], g["scale"], g["out_scale"], g["loss_weight"])
    _, g0, _ = C.loss_and_grad(params, m, y, *args, rounding=False)
    _, g1, _ = C.loss_and_grad(params, m, y, *args, rounding=True)
    rel = np.linalg.norm(g1 - g0) / np.linalg.norm(g0)
    assert 1e-5 < rel < 3e-2


def test_adam_constant_gradient_closed_form():
    """Under a constant gradient g every bias-corrected Adam step moves by -lr g / (|g| + eps)."""
    rng = np.random.default_rng(6)
    p0 = rng.normal(size=50)
    g = rng.normal(size=50)
    p, mo, ve = p0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 4):
        p_new, mo, ve = C.adam_step(p, g, mo, ve, step, lr=1e-3)
        assert np.allclose(p_new - p, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=0)
        p = p_new


def test_restriction_identities():
    k, r, R = 4, 1.0, 2.5
    Hf, Wf = 32, 48
    J = C.torus_J(r, R, Hf)
    # constants are kept
    c = C.restrict(np.full((Hf, Wf), 1.7), k, J)
    assert np.allclose(c, 1.7, rtol=0, atol=1e-14)
    # J-weighted totals carry over: sum_Q W_Q sum_S c = (1/k) sum_{q,s} J_q f
    rng = np.random.default_rng(7)
    f = rng.normal(size=(Hf, Wf))
    c = C.restrict(f, k, J)
    d, w = C.fine_weights(k)
    WQ = np.array([sum(ww * J[(k * Q + dd) % Hf] for dd, ww in zip(d, w)) for Q in range(Hf // k)])
    assert abs(np.sum(WQ[:, None] * c) - np.sum(J[:, None] * f) / k) < 1e-12 * np.abs(f).sum()
    # Fourier symbol of full weighting along phi: cos(m phi) -> cos(m phi) (1 + 2 cos mh + cos 2mh)/4
    ph = 2 * np.pi * np.arange(Wf) / Wf
    h = 2 * np.pi / Wf
    for mode in (1, 3, 5):
        c = C.restrict(np.cos(mode * ph)[None, :].repeat(Hf, 0), k, J)
        sym = (1 + 2 * math.cos(mode * h) + math.cos(2 * mode * h)) / 4
        assert np.allclose(c, sym * np.cos(mode * ph[::k])[None, :], rtol=0, atol=1e-13)


def test_correction_moment_identities():
    rng = np.random.default_rng(8)
    H, W, r, R = 6, 10, 1.0, 2.5
    n = 1 + 0.05 * rng.uniform(-1, 1, (H, W))
    ut, up = 0.05 * rng.uniform(-1, 1, (2, H, W))
    f = C.feq(n, ut, up) * (1 + 0.01 * rng.uniform(-1, 1, (16, H, W)))
    phi = rng.uniform(-1, 1, (H, W))
    delta = rng.normal(size=(H, W, 4)) * np.array([1e-2, 1e-3, 1e-3, 1e-3])
    f2, phi2 = C.apply_correction(f, phi, delta, r, R)
    J = C.torus_J(r, R, H)[:, None]
    n0, u0t, u0p = C.moments(f)
    n1, u1t, u1p = C.moments(f2)
    dn = delta[..., 1] - np.sum(J * delta[..., 1]) / (np.sum(J) * W)
    assert np.allclose(n1, n0 + dn, rtol=0, atol=1e-14)
    assert np.allclose(u1t, u0t + delta[..., 2], rtol=0, atol=1e-14)
    assert np.allclose(u1p, u0p + delta[..., 3], rtol=0, atol=1e-14)
    assert abs(np.sum(J * n1) - np.sum(J * n0)) < 1e-13 * np.sum(J * n0)
    assert abs(np.sum(J * phi2) - np.sum(J * phi)) < 1e-13 * np.sum(J)
    f3, phi3 = C.apply_correction(f, phi, np.zeros((H, W, 4)), r, R)
    assert np.allclose(f3, f, rtol=1e-15, atol=0) and np.array_equal(phi3, phi)

