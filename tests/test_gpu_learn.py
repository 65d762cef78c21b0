"""GPU parity of the learned coarse-step correction: the HIP kernels of tlb_learn.h (matrix-core
convolutions, back-propagation, Adam, restriction, moments/targets, correction, learned step)
against the numpy reference oracle/cnn_ref.py and the C oracle, on seeded inputs.

Tolerances.  Both sides round the same operands to bfloat16 at the same points; they differ
in accumulation (FP32 on the matrix cores against exact FP64 sums): about 1e-6 relative before
each rounding, which flips a bfloat16 rounding (2^-8 relative) for a fraction of order 1e-3 of
the hidden values.  Propagated to the output that is a relative L2 difference of order 1e-4;
the bars are 1e-3 (L2) and 1e-2 (L-infinity, relative to the largest value).  Operations
without bfloat16 (restriction, moments, correction) are held to FP64 / FP32 rounding.
"""

import numpy as np
import pytest

from paper_1904_10070_amd import inputs
from oracle import cnn_ref as C

pytestmark = pytest.mark.gpu

GEO = dict(r=1.0, R=2.5)
SHIFT = (0.0, 1.0, 0.0, 0.0)
SCALE = (1.0, 50.0, 100.0, 100.0)
OUT_SCALE = (1e-3, 1e-6, 1e-5, 1e-5)
LOSS_W = (2.0, 1.0, 0.5, 0.5)


def rel_l2(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def rel_linf(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def make_net(torch, H, W, max_batch, params):
    from paper_1904_10070_amd.binding import CoarseCNN
    net = CoarseCNN(GEO["r"], GEO["R"], H, W, max_batch, SHIFT, SCALE, OUT_SCALE, LOSS_W)
    net.set_params(params)
    return net


def params_with_biases(seed):
    p = inputs.cnn_init_params(seed, last_gain=1.0)
    rng = np.random.default_rng(seed + 100)
    return (p + 0.02 * rng.normal(size=p.shape)).astype(np.float32)


@pytest.mark.parametrize("shape", [(12, 40), (7, 64), (5, 19)])
def test_forward_matches_reference(torch_cuda, shape):
    """Ragged rows (40 = 2 x 16 + 8, 19 < 64), a single full strip (64), odd theta counts."""
    torch = torch_cuda
    H, W = shape
    params = params_with_biases(1)
    m, _ = inputs.learn_samples(2, 3, H, W)
    net = make_net(torch, H, W, 3, params)
    idx = [2, 0, 1]
    out = net.forward(torch.tensor(m, device="cuda"), idx=idx).cpu().numpy().astype(np.float64)
    _, z = C.forward(params.astype(np.float64), m[idx].astype(np.float64), GEO["r"], GEO["R"],
                     SHIFT, SCALE)
    ref = z * np.array(OUT_SCALE)
    e2, ei = rel_l2(out, ref), rel_linf(out, ref)
    print(f"forward {H}x{W}: rel L2 {e2:.2e}, rel Linf {ei:.2e}", flush=True)
    assert e2 <= 1e-3 and ei <= 1e-2


def test_forward_more_samples_than_a_grid_dimension(torch_cuda):
    """66000 samples of a 1 x 2 torus: more batch slots than a launch grid's second or third
    dimension holds (65535), every tap wrapping onto the row's two nodes."""
    torch = torch_cuda
    n, H, W = 66000, 1, 2
    params = params_with_biases(13)
    m, _ = inputs.learn_samples(14, n, H, W)
    net = make_net(torch, H, W, n, params)
    out = net.forward(torch.tensor(m, device="cuda")).cpu().numpy().astype(np.float64)
    _, z = C.forward(params.astype(np.float64), m.astype(np.float64), GEO["r"], GEO["R"], SHIFT, SCALE)
    ref = z * np.array(OUT_SCALE)
    e2, ei = rel_l2(out, ref), rel_linf(out, ref)
    print(f"forward {n}x{H}x{W}: rel L2 {e2:.2e}, rel Linf {ei:.2e}", flush=True)
    assert e2 <= 1e-3 and ei <= 1e-2


def test_forward_full_coarse_grid(torch_cuda):
    """The 128 x 320 coarse grid the learned step runs on, one sample, all outputs."""
    torch = torch_cuda
    H, W = 128, 320
    params = params_with_biases(3)
    m, _ = inputs.learn_samples(4, 1, H, W)
    net = make_net(torch, H, W, 1, params)
    out = net.forward(torch.tensor(m, device="cuda")).cpu().numpy().astype(np.float64)
    _, z = C.forward(params.astype(np.float64), m.astype(np.float64), GEO["r"], GEO["R"], SHIFT, SCALE)
    ref = z * np.array(OUT_SCALE)
    e2, ei = rel_l2(out, ref), rel_linf(out, ref)
    print(f"forward 128x320: rel L2 {e2:.2e}, rel Linf {ei:.2e}", flush=True)
    assert e2 <= 1e-3 and ei <= 1e-2


@pytest.mark.parametrize("shape", [(12, 40), (6, 70)])
def test_gradient_matches_reference(torch_cuda, shape):
    """Loss and the gradient of every layer's weights and biases (ragged strips of 64)."""
    torch = torch_cuda
    H, W = shape
    params = params_with_biases(5)
    m, y = inputs.learn_samples(6, 4, H, W)
    net = make_net(torch, H, W, 3, params)
    idx = [3, 1, 2]
    loss, grad = net.gradient(torch.tensor(m, device="cuda"), torch.tensor(y, device="cuda"), idx=idx)
    L, g_ref, _ = C.loss_and_grad(params.astype(np.float64), m[idx].astype(np.float64),
                                  y[idx].astype(np.float64), GEO["r"], GEO["R"], SHIFT, SCALE,
                                  OUT_SCALE, LOSS_W)
    assert abs(loss - L) <= 1e-4 * L, (loss, L)
    o = 0
    for l, (ci, co) in enumerate(C.ARCH):
        nW = co * 9 * ci
        for name, sl in (("W", slice(o, o + nW)), ("b", slice(o + nW, o + nW + co))):
            e = rel_l2(grad[sl].astype(np.float64), g_ref[sl])
            print(f"layer {l} d{name}: rel L2 {e:.2e}", flush=True)
            assert e <= 1e-3, (l, name, e)
        o += nW + co


@pytest.mark.parametrize("shape", [(8, 64, 136), (6, 48, 200), (32, 2, 832), (32, 1, 1600)])
def test_forward_and_gradient_with_many_tiles_per_wavefront(torch_cuda, shape):
    """More 64-node strips (1536, 1152, 832, 800) than weight-gradient workgroups and more
    16-node tiles (4608, 3744, 3328, 3200) than convolution wavefronts on this part, so that
    each walks several strips or tiles, carrying across rows and samples, with ragged row ends
    (136 = 2 x 64 + 8, 200 = 3 x 64 + 8); with one or two rows the window of input rows and the
    taps carried to the next row wrap onto themselves."""
    torch = torch_cuda
    n, H, W = shape
    params = params_with_biases(11)
    m, y = inputs.learn_samples(12, n, H, W)
    net = make_net(torch, H, W, n, params)
    mt, yt = torch.tensor(m, device="cuda"), torch.tensor(y, device="cuda")
    out = net.forward(mt).cpu().numpy().astype(np.float64)
    _, z = C.forward(params.astype(np.float64), m.astype(np.float64), GEO["r"], GEO["R"], SHIFT, SCALE)
    ref = z * np.array(OUT_SCALE)
    e2, ei = rel_l2(out, ref), rel_linf(out, ref)
    print(f"forward {n}x{H}x{W}: rel L2 {e2:.2e}, rel Linf {ei:.2e}", flush=True)
    assert e2 <= 1e-3 and ei <= 1e-2
    loss, grad = net.gradient(mt, yt)
    L, g_ref, _ = C.loss_and_grad(params.astype(np.float64), m.astype(np.float64),
                                  y.astype(np.float64), GEO["r"], GEO["R"], SHIFT, SCALE,
                                  OUT_SCALE, LOSS_W)
    assert abs(loss - L) <= 1e-4 * L, (loss, L)
    o = 0
    for l, (ci, co) in enumerate(C.ARCH):
        nW = co * 9 * ci
        for name, sl in (("W", slice(o, o + nW)), ("b", slice(o + nW, o + nW + co))):
            e = rel_l2(grad[sl].astype(np.float64), g_ref[sl])
            print(f"layer {l} d{name}: rel L2 {e:.2e}", flush=True)
            assert e <= 1e-3, (l, name, e)
        o += nW + co


def test_gradient_close_to_exact_network(torch_cuda):
    """Against the exact network (no rounding), whose gradient the oracle pins by finite
    differences: the bfloat16 policy costs about 1 % of the gradient."""
    torch = torch_cuda
    H, W = 10, 32
    params = params_with_biases(7)
    m, y = inputs.learn_samples(8, 2, H, W)
    net = make_net(torch, H, W, 2, params)
    _, grad = net.gradient(torch.tensor(m, device="cuda"), torch.tensor(y, device="cuda"))
    _, g0, _ = C.loss_and_grad(params.astype(np.float64), m.astype(np.float64),
                               y.astype(np.float64), GEO["r"], GEO["R"], SHIFT, SCALE,
                               OUT_SCALE, LOSS_W, rounding=False)
    e = rel_l2(grad.astype(np.float64), g0)
    print(f"gradient vs exact network: rel L2 {e:.2e}", flush=True)
    assert e <= 3e-2


def test_adam_step_matches_reference(torch_cuda):
    torch = torch_cuda
    H, W = 8, 48
    params = params_with_biases(9)
    m, y = inputs.learn_samples(10, 2, H, W)
    net = make_net(torch, H, W, 2, params)
    mt, yt = torch.tensor(m, device="cuda"), torch.tensor(y, device="cuda")
    p = params.astype(np.float64)
    mo, ve = np.zeros_like(p), np.zeros_like(p)
    for step in (1, 2, 3):
        _, g_ref, _ = C.loss_and_grad(p, m.astype(np.float64), y.astype(np.float64), GEO["r"],
                                      GEO["R"], SHIFT, SCALE, OUT_SCALE, LOSS_W)
        p_next, mo, ve = C.adam_step(p, g_ref, mo, ve, step, lr=1e-3)
        net.train_step(mt, yt, [0, 1], step, 1e-3)
        got = net.get_params().astype(np.float64)
        upd_ref, upd = p_next - p, got - p
        e = rel_l2(upd, upd_ref)
        frac = np.mean(np.abs(upd - upd_ref) > 0.05e-3)
        print(f"adam step {step}: update rel L2 {e:.2e}, entries off by > 5% of lr: {frac:.2e}",
              flush=True)
        assert e <= 2e-2 and frac <= 1e-2
        p = got      # follow the GPU's weights so that differences do not accumulate


@pytest.mark.parametrize("precision, density", [(64, 1.0), (32, 1.0), (32, 20.0)])
def test_restrict_matches_reference(torch_cuda, precision, density):
    """(density 20: the FP32 coarse grid takes over the fine grid's reference density)"""
    from paper_1904_10070_amd import TorusGrid
    from paper_1904_10070_amd.binding import restrict
    pf = inputs.TorusParams(1.0, 2.5, 32, 80, 0.5, 2e-3, 0.05, 0.3, 2e-4)
    pc = pf.with_(n_theta=8, n_phi=20)
    f, phi = inputs.random_populations(32, 80, seed=11)
    f = density * f
    fine, coarse = TorusGrid(pf, precision), TorusGrid(pc, precision)
    fine.set_state(phi, f=f)
    restrict(fine, coarse)
    fc, phic = (x.double().cpu().numpy() for x in coarse.get_state())
    f_ref, phi_ref = C.restrict_state(f, phi, 4, 1.0, 2.5)
    tol = 1e-14 if precision == 64 else 2e-7
    assert rel_linf(fc, f_ref) <= tol and rel_linf(phic, phi_ref) <= tol


def test_pair_and_correction_match_reference(torch_cuda):
    torch = torch_cuda
    from paper_1904_10070_amd import TorusGrid
    from paper_1904_10070_amd.binding import learn_pair, apply_correction
    p = inputs.TorusParams(1.0, 2.5, 12, 36, 0.5, 2e-3, 0.05, 0.3, 2e-4)
    fa, pa = inputs.random_populations(12, 36, seed=12)
    fb, pb = inputs.random_populations(12, 36, seed=13)
    ga, gb = TorusGrid(p, 64), TorusGrid(p, 64)
    ga.set_state(pa, f=fa)
    gb.set_state(pb, f=fb)
    m, y = learn_pair(ga, gb)
    ma, mb = C.moment_fields(fa, pa), C.moment_fields(fb, pb)
    assert rel_linf(m.cpu().numpy().astype(np.float64), ma) <= 1e-7
    for c in range(4):
        assert rel_linf(y.cpu().numpy()[..., c].astype(np.float64), (mb - ma)[..., c]) <= 1e-7
    rng = np.random.default_rng(14)
    delta = (rng.normal(size=(12, 36, 4)) * np.array([1e-2, 1e-3, 1e-3, 1e-3])).astype(np.float32)
    apply_correction(ga, torch.tensor(delta, device="cuda"))
    f2, phi2 = (x.cpu().numpy() for x in ga.get_state())
    f_ref, phi_ref = C.apply_correction(fa, pa, delta.astype(np.float64), 1.0, 2.5)
    assert rel_linf(f2, f_ref) <= 1e-13 and rel_linf(phi2, phi_ref) <= 1e-13


def test_learned_step_matches_reference(torch_cuda):
    """One learned step on an FP64 coarse grid: the C oracle's step, the reference network and
    the reference correction, against tlb_learned_step_n."""
    torch = torch_cuda
    from paper_1904_10070_amd import TorusGrid
    from paper_1904_10070_amd.binding import learned_step
    from tests.helpers import oracle_run
    p = inputs.TorusParams(1.0, 2.5, 16, 48, 0.5, 2e-3, 0.05, 0.3, 2e-4)
    phi, n, ut, up = inputs.random_state(p, seed=15)
    params = params_with_biases(16)
    net = make_net(torch, 16, 48, 1, params)
    g = TorusGrid(p, 64)
    g.set_state(phi, n, ut, up)
    learned_step(g, net, 1)
    f_gpu, phi_gpu = (x.cpu().numpy() for x in g.get_state())
    og, f1, phi1 = oracle_run(p, phi, n, ut, up, 1)
    m = C.moment_fields(f1, phi1)[None]
    _, z = C.forward(params.astype(np.float64), m, 1.0, 2.5, SHIFT, SCALE)
    f_ref, phi_ref = C.apply_correction(f1, phi1, z[0] * np.array(OUT_SCALE), 1.0, 2.5)
    # the state differs from the reference by the network's output difference (bar: 1 % of
    # the largest output) times the size of the correction it drives
    ef, ep = np.abs(f_gpu - f_ref).max(), np.abs(phi_gpu - phi_ref).max()
    cf, cp = np.abs(f_ref - f1).max(), np.abs(phi_ref - phi1).max()
    print(f"learned step: |df| {ef:.2e} of correction {cf:.2e}; |dphi| {ep:.2e} of {cp:.2e}",
          flush=True)
    assert cf > 0 and cp > 0
    assert ef <= 1e-2 * cf + 1e-14 and ep <= 1e-2 * cp + 1e-14


@pytest.mark.parametrize("precision,shape", [(64, (16, 48)), (64, (13, 29)), (64, (5, 19)),
                                               (64, (24, 72)), (32, (40, 100))])
def test_learned_step_network_equals_layer_by_layer(torch_cuda, precision, shape):
    """tlb_learned_step_n runs the network in one launch (8 x 24 tiles with a five-node halo,
    activations in LDS); the public calls run it layer by layer (tlb_learn_pair,
    tlb_cnn_forward, tlb_apply_correction).  Both make the same products in the same order
    with the same bfloat16 roundings, so the network outputs agree bit for bit, and the states
    after a step differ only by the summation order of the area-weighted mean correction
    (rounding of the FP64 sums, FP64 grids) and by where the order parameter is folded into
    its base (FP32 grids).  Shapes: several tiles with ragged edges, a grid smaller than one
    tile in both directions (wrap-around halo), an exact multiple of the tile."""
    torch = torch_cuda
    from paper_1904_10070_amd import TorusGrid
    from paper_1904_10070_amd.binding import learned_step, learn_pair, apply_correction
    H, W = shape
    p = inputs.TorusParams(1.0, 2.5, H, W, 0.5, 2e-3, 0.05, 0.3, 2e-4)
    state = inputs.random_state(p, seed=31)
    net = make_net(torch, H, W, 1, params_with_biases(32))
    a, b = TorusGrid(p, precision), TorusGrid(p, precision)
    for g in (a, b):
        g.set_state(*state)
    learned_step(a, net, 1)
    b.step(1)
    m, _ = learn_pair(b)
    z = net.forward(m[None])
    apply_correction(b, z[0].contiguous())   # tlb_cnn_forward returns z * out_scale
    fa, pa = (x.cpu().numpy().astype(np.float64) for x in a.get_state())
    fb, pb = (x.cpu().numpy().astype(np.float64) for x in b.get_state())
    # the size of the correction: the step without it
    c = TorusGrid(p, precision)
    c.set_state(*state)
    c.step(1)
    f1, p1 = (x.cpu().numpy().astype(np.float64) for x in c.get_state())
    cf, cp = np.abs(fb - f1).max(), np.abs(pb - p1).max()
    ef, ep = np.abs(fa - fb).max(), np.abs(pa - pb).max()
    print(f"{precision} {shape}: |df| {ef:.2e} of correction {cf:.2e}; |dphi| {ep:.2e} of {cp:.2e}",
          flush=True)
    assert cf > 0 and cp > 0
    if precision == 64:
        assert ef <= 1e-12 * cf and ep <= 1e-12 * cp
    else:  # a few FP32 roundings of f (~0.1) and phi (~1)
        assert ef <= 3e-8 and ep <= 3e-7


def test_learned_step_graph_is_bitwise(torch_cuda):
    """40 learned steps as one 32-step graph replay plus 8 plain steps, against 40 plain."""
    torch = torch_cuda
    from paper_1904_10070_amd import TorusGrid, NO_GRAPH
    from paper_1904_10070_amd.binding import learned_step
    p = inputs.TorusParams(1.0, 2.5, 16, 48, 0.5, 2e-3, 0.05, 0.3, 2e-4)
    phi, n, ut, up = inputs.random_state(p, seed=17)
    params = (inputs.cnn_init_params(18) * 0.3).astype(np.float32)
    net = make_net(torch, 16, 48, 1, params)
    a, b = TorusGrid(p, 32), TorusGrid(p.with_(flags=NO_GRAPH), 32)
    for g in (a, b):
        g.set_state(phi, n, ut, up)
    for call in range(3):
        learned_step(a, net, 40)
        learned_step(b, net, 40)
        torch.cuda.synchronize()
        fa, pa = a.get_state()
        fb, pb = b.get_state()
        assert torch.equal(fa, fb) and torch.equal(pa, pb), call
        assert torch.isfinite(fa).all()


def test_learned_step_graph_not_reused_by_a_new_grid(torch_cuda):
    """The learned-step graph keeps the stage arguments of the grid it was built for.  A grid
    created after that one was destroyed, on the very same state buffers (and often at the same
    host address) but with another tau and dt, must not replay it: 40 learned steps of the new
    grid equal 40 plain-launch steps (TLB_NO_GRAPH) of a grid with its parameters, bit for bit."""
    torch = torch_cuda
    from paper_1904_10070_amd import TorusGrid, NO_GRAPH
    from paper_1904_10070_amd.binding import learned_step
    p = inputs.TorusParams(1.0, 2.5, 16, 48, 0.5, 2e-3, 0.05, 0.3, 2e-4)
    q = p.with_(tau=0.7, dt=1.5e-4)
    phi, n, ut, up = inputs.random_state(p, seed=19)
    params = (inputs.cnn_init_params(20) * 0.3).astype(np.float32)
    net = make_net(torch, 16, 48, 1, params)
    a = TorusGrid(p, 32)
    a.set_state(phi, n, ut, up)
    learned_step(a, net, 40)                    # builds the graph for grid a
    bufs = (a.f, a.phi)
    a.close()
    b = TorusGrid(q, 32, buffers=bufs)          # same buffers, other parameters
    b.set_state(phi, n, ut, up)
    learned_step(b, net, 40)
    c = TorusGrid(q.with_(flags=NO_GRAPH), 32)
    c.set_state(phi, n, ut, up)
    learned_step(c, net, 40)
    torch.cuda.synchronize()
    fb, pb = b.get_state()
    fc, pc = c.get_state()
    assert torch.equal(fb, fc) and torch.equal(pb, pc)
