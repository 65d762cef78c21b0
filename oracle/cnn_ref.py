"""Plain numpy (FP64) reference of the learned coarse-step correction.

TEST INFRASTRUCTURE ONLY: the CPU reference that the HIP learning kernels are checked
against.  Only tests, the smoke check and the benchmark's CPU-baseline leg may import it.  It
imports nothing from the GPU package.

What is defined here (the learned part extends the paper's method; the torus, its metric
factor J = R + r cos(theta) and the equilibrium come from section II, eqs. torus and feq):

* the network: five periodic 3x3 convolutions, widths 6 -> 32 -> 32 -> 32 -> 32 -> 4, ReLU
  between them.  Inputs per node: (phi, n, u_theta, u_phi) shifted and scaled, r and
  R + r cos(theta).  Outputs: corrections (dphi, dn, du_theta, du_phi) in units of
  `out_scale`.  Tap t = 3 (dy + 1) + (dx + 1) reads the node (y + dy, x + dx), y along theta
  and x along phi, both periodic.
* its precision policy (what the GPU kernels store in bfloat16): the input features, the
  weights as used by the products, the hidden activations and the back-propagated error
  signals are rounded to bfloat16 (round to nearest even); products accumulate exactly here
  (FP64) and in FP32 on the GPU; biases, the last layer's output and the loss stay wide.
  `rounding=False` turns every rounding off (the exact network, for finite differences).
* the loss L = sum_c w_c (z_c - y_c / s_c)^2 / (N H W 4) and its gradient with respect to
  the FP32 master weights (straight through the bfloat16 rounding of the weights);
* one Adam step;
* the restriction of a fine torus state to a grid coarser by an integer factor k: full
  weighting, 1/2 at the two end nodes of a 2k-wide stencil and 1 inside, J-weighted along theta
  so that sum_Q W_Q c_Q = sum_q J_q f_q with W_Q the row weight (J-weighted mass carries
  over exactly);
* the correction of a coarse state: the J-weighted means of dphi and dn are removed (so mass
  and sum_J phi stay fixed), then f += f_eq(n + dn, u + du) - f_eq(n, u) and phi += dphi.

Parameters are one flat FP32 vector, layer by layer: W[c_out][tap][c_in] then b[c_out].
"""

import numpy as np

from .flat_numpy import velocity_set

ARCH = ((6, 32), (32, 32), (32, 32), (32, 32), (32, 4))
TAPS = tuple((t // 3 - 1, t % 3 - 1) for t in range(9))   # (dy, dx) of tap t


# -- parameters --------------------------------------------------------------------------------

def param_count(arch=ARCH):
    return sum(co * 9 * ci + co for ci, co in arch)


def unpack(params, arch=ARCH):
    out, o = [], 0
    for ci, co in arch:
        W = np.asarray(params[o:o + co * 9 * ci], dtype=np.float64).reshape(co, 9, ci)
        o += co * 9 * ci
        b = np.asarray(params[o:o + co], dtype=np.float64)
        o += co
        out.append((W, b))
    assert o == len(params)
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


# -- bfloat16 ----------------------------------------------------------------------------------

def bf16(x):
    """Round to the nearest bfloat16 (ties to even), through the FP32 value; finite inputs."""
    b = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32)).view(np.uint32)
    b = (b + np.uint32(0x7FFF) + ((b >> np.uint32(16)) & np.uint32(1))) & np.uint32(0xFFFF0000)
    return b.view(np.float32).astype(np.float64)


# -- periodic 3x3 convolution and its two adjoints -----------------------------------------------

def conv3x3(a, W, b=None):
    """z[n, y, x, o] = b[o] + sum_t sum_i W[o, t, i] a[n, y + dy_t, x + dx_t, i] (periodic)."""
    N, H, Wd, _ = a.shape
    z = np.zeros((N, H, Wd, W.shape[0]))
    for t, (dy, dx) in enumerate(TAPS):
        s = np.roll(a, shift=(-dy, -dx), axis=(1, 2))    # s[:, y, x] = a[:, y + dy, x + dx]
        z += s @ W[:, t, :].T
    if b is not None:
        z += b
    return z


def conv3x3_transpose(e, W):
    """Adjoint of conv3x3 in its input: g[n, y, x, i] = sum_t sum_o W[o, t, i] e[n, y - dy, x - dx, o]."""
    N, H, Wd, _ = e.shape
    g = np.zeros((N, H, Wd, W.shape[2]))
    for t, (dy, dx) in enumerate(TAPS):
        s = np.roll(e, shift=(dy, dx), axis=(1, 2))      # s[:, y, x] = e[:, y - dy, x - dx]
        g += s @ W[:, t, :]
    return g


def conv3x3_weight_grad(e, a):
    """Adjoint of conv3x3 in its weights: dW[o, t, i] = sum_{n,y,x} e[n, y, x, o] a[n, y + dy, x + dx, i]."""
    out = np.zeros((e.shape[3], 9, a.shape[3]))
    for t, (dy, dx) in enumerate(TAPS):
        s = np.roll(a, shift=(-dy, -dx), axis=(1, 2))
        out[:, t, :] = np.einsum("nyxo,nyxi->oi", e, s)
    return out


# -- the network ---------------------------------------------------------------------------------

def features(m, r, R, shift, scale, rounding=True):
    """m: [N, H, W, 4] raw (phi, n, u_theta, u_phi) -> [N, H, W, 6] network input."""
    N, H, Wd, _ = m.shape
    theta = 2.0 * np.pi * np.arange(H) / H
    x = np.zeros((N, H, Wd, 6))
    x[..., :4] = (m - np.asarray(shift, dtype=np.float64)) * np.asarray(scale, dtype=np.float64)
    x[..., 4] = r
    x[..., 5] = (R + r * np.cos(theta))[None, :, None]
    return bf16(x) if rounding else x


def forward(params, m, r, R, shift, scale, rounding=True, arch=ARCH):
    """Returns (activations [x, a_0, .., a_3], z_4) with z_4 the last layer's wide output."""
    layers = unpack(params, arch)
    rnd = bf16 if rounding else (lambda v: v)
    acts = [features(m, r, R, shift, scale, rounding)]
    for l, (W, b) in enumerate(layers):
        z = conv3x3(acts[-1], rnd(W), b)
        if l == len(layers) - 1:
            return acts, z
        acts.append(rnd(np.maximum(z, 0.0)))


def loss_and_grad(params, m, y, r, R, shift, scale, out_scale, loss_weight, rounding=True,
                  arch=ARCH):
    """Loss L = sum w_c (z_c - y_c / s_c)^2 / (N H W 4) and dL/dparams (flat, FP64)."""
    layers = unpack(params, arch)
    rnd = bf16 if rounding else (lambda v: v)
    acts, z = forward(params, m, r, R, shift, scale, rounding, arch)
    w = np.asarray(loss_weight, dtype=np.float64)
    d = z - y / np.asarray(out_scale, dtype=np.float64)
    count = d.size
    L = float(np.sum(w * d * d) / count)
    e = rnd(w * d)                      # error signal of the last layer (dL/dz * count / 2)
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        dW = conv3x3_weight_grad(e, acts[l]) * (2.0 / count)
        db = e.sum(axis=(0, 1, 2)) * (2.0 / count)
        grads[l] = (dW, db)
        if l > 0:
            e = rnd(conv3x3_transpose(e, rnd(W)) * (acts[l] > 0))
    return L, pack(grads), z


def adam_step(params, grad, mom, vel, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015, algorithm 1); step counts from 1.  Returns new arrays."""
    mom = beta1 * mom + (1 - beta1) * grad
    vel = beta2 * vel + (1 - beta2) * grad * grad
    mhat = mom / (1 - beta1 ** step)
    vhat = vel / (1 - beta2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), mom, vel


# -- torus state: moments, restriction, correction ----------------------------------------------

def torus_J(r, R, n_theta):
    return R + r * np.cos(2.0 * np.pi * np.arange(n_theta) / n_theta)


def moments(f):
    """f: [16, H, W], population k = 4 i + j -> (n, u_theta, u_phi) with n u = sum f v."""
    v, _, _ = velocity_set()
    fk = f.reshape(4, 4, *f.shape[1:])
    n = f.sum(axis=0)
    ut = np.einsum("i,ij...->...", v, fk) / n
    up = np.einsum("j,ij...->...", v, fk) / n
    return n, ut, up


def feq(n, ut, up):
    """Third-order Hermite equilibrium (section II, eq. feq) with k_B T = m = 1."""
    v, w, _ = velocity_set()
    vi = v[:, None, None, None]
    vj = v[None, :, None, None]
    xi = vi * ut + vj * up
    u2 = ut * ut + up * up
    ww = (w[:, None] * w[None, :])[:, :, None, None]
    out = n * ww * (1 + xi + 0.5 * (xi * xi - u2) + xi * (xi * xi - 3 * u2) / 6)
    return out.reshape(16, *n.shape)


def fine_weights(k):
    """Full-weighting stencil of a factor-k restriction: offsets -k/2..k/2, 1/2 at the ends."""
    assert k % 2 == 0
    d = np.arange(-k // 2, k // 2 + 1)
    w = np.ones(len(d))
    w[0] = w[-1] = 0.5
    return d, w


def restrict(field, k, J_fine):
    """field [..., H_f, W_f] -> [..., H_f / k, W_f / k]: J-weighted full weighting in theta,
    plain full weighting in phi (both periodic)."""
    Hf, Wf = field.shape[-2:]
    assert Hf % k == 0 and Wf % k == 0
    d, w = fine_weights(k)
    Jb = np.broadcast_to(J_fine[:, None], (Hf, Wf))
    num = np.zeros(field.shape[:-2] + (Hf // k, Wf))
    den = np.zeros((Hf // k, Wf))
    for dd, ww in zip(d, w):
        rows = (np.arange(Hf // k) * k + dd) % Hf
        num += ww * (Jb * field)[..., rows, :]
        den += ww * Jb[rows, :]
    col = num / den
    out = np.zeros(field.shape[:-2] + (Hf // k, Wf // k))
    for dd, ww in zip(d, w):
        cols = (np.arange(Wf // k) * k + dd) % Wf
        out += ww * col[..., cols]
    return out / w.sum()


def restrict_state(f, phi, k, r, R):
    J = torus_J(r, R, f.shape[1])
    return restrict(f, k, J), restrict(phi, k, J)


def moment_fields(f, phi):
    """[H, W, 4] = (phi, n, u_theta, u_phi), the network's raw input and target layout."""
    n, ut, up = moments(f)
    return np.stack([phi, n, ut, up], axis=-1)


def apply_correction(f, phi, delta, r, R):
    """delta [H, W, 4] = (dphi, dn, du_theta, du_phi) in physical units."""
    J = torus_J(r, R, f.shape[1])[:, None]
    dphi = delta[..., 0] - np.sum(J * delta[..., 0]) / (np.sum(J) * delta.shape[1])
    dn = delta[..., 1] - np.sum(J * delta[..., 1]) / (np.sum(J) * delta.shape[1])
    n, ut, up = moments(f)
    f_new = f + feq(n + dn, ut + delta[..., 2], up + delta[..., 3]) - feq(n, ut, up)
    return f_new, phi + dphi
