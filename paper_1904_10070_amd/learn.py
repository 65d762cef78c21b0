"""Learned coarse step: training data from the solver, training, and evaluation judged by the
fine solver.  Host logic only: every field operation runs in libtlb's kernels (tlb.h and
tlb_learn.h); this module orders the calls and keeps the bookkeeping.

Workflow (spinodal coarsening on the torus, section IV of the paper):
  * a fine grid runs the plain scheme; at each sample time its state is restricted onto a
    coarse grid k times coarser (tlb_restrict), the coarse grid takes one step of dt_factor
    times the fine time step, the fine grid takes dt_factor steps and is restricted again;
    the sample is (moments of the stepped coarse state, restricted fine moments minus them)
    (tlb_learn_pair);
  * the network is trained on these pairs by the library's own forward / backward / Adam
    kernels (tlb_cnn_train_step);
  * evaluation hands a fine state over to the coarse grid at t_start and runs the learned
    coarse step (tlb_learned_step_n) and the plain coarse step side by side, with the fine
    solver continuing as the judge: the coarsening length L_d = A_total / L_I (section IV,
    eq. cart_scaling_L0) of each coarse state against that of the restricted fine state, and
    the relative L2 difference of phi.
"""
import math
import time

import numpy as np

from . import inputs
from .binding import (TorusGrid, CoarseCNN, restrict, learn_pair, learned_step, learn_stats,
                      apply_correction)


def coarse_params(p_fine, k=4, dt_factor=4, **override):
    """The coarse grid: n_theta / k x n_phi / k nodes, time step dt_factor x the fine one,
    the same physical parameters (so the fine interface width) unless overridden."""
    assert p_fine.n_theta % k == 0 and p_fine.n_phi % k == 0
    return p_fine.with_(n_theta=p_fine.n_theta // k, n_phi=p_fine.n_phi // k,
                        dt=p_fine.dt * dt_factor, **override)


def _steps(t, dt):
    return int(round(t / dt))


def coarse_grid(pc, precision=32):
    """A coarse grid with the stage kernel's tile height chosen by the autotuner (small grids
    prefer short tiles: more workgroups in flight)."""
    g = TorusGrid(pc, precision)
    g.tile_rows = g.autotune()
    return g


def generate_pairs(p_fine, seeds, t_first, t_last, every, k=4, dt_factor=4, precision=32,
                   coarse_override=None, noise=None, net=None, leads=(0,), reject=None,
                   progress=print):
    """Training pairs from fine spinodal runs (one per seed): a sample every `every` fine
    steps for t in [t_first, t_last].  Returns float32 device tensors (m, y), each
    [samples, n_theta / k, n_phi / k, 4].

    noise = (sigma_phi, sigma_n, sigma_u) perturbs every other restricted state (through
    tlb_apply_correction) before its coarse step, with the target still the restricted fine
    state: such pairs teach the network to pull a drifted coarse state back.  The noise is
    drawn from a seeded device generator.

    leads (cycled over the samples, each > 0 needs `net`): the restricted state first takes
    that many learned coarse steps while the fine grid keeps pace, and the pair is formed from
    there -- inputs drawn from the learned model's own drift, targets still the fine truth
    (pushforward training).  Such a pair is dropped if the state turned non-finite or, with
    reject = (scale[4], limit), if the RMS of a target channel with nonzero scale exceeds
    limit x scale (a zero scale leaves the channel unchecked)."""
    import torch
    assert every >= (max(leads) + 1) * dt_factor
    assert net is not None or max(leads) == 0
    gen = None
    if noise is not None:
        gen = torch.Generator(device="cuda")
        gen.manual_seed(int(1000 + sum(seeds)))
    pc = coarse_params(p_fine, k, dt_factor, **(coarse_override or {}))
    per_seed = (_steps(t_last, p_fine.dt) - _steps(t_first, p_fine.dt)) // every + 1
    shape = (len(seeds) * per_seed, pc.n_theta, pc.n_phi, 4)
    m = torch.empty(shape, dtype=torch.float32, device="cuda")
    y = torch.empty(shape, dtype=torch.float32, device="cuda")
    ca, cb = TorusGrid(pc, precision), TorusGrid(pc, precision)
    i = 0
    for seed in seeds:
        t0 = time.time()
        fine = TorusGrid(p_fine, precision)
        fine.set_state(inputs.spinodal_phi(p_fine, seed=seed),
                       *inputs.rest_moments(p_fine.n_theta, p_fine.n_phi))
        fine.step(_steps(t_first, p_fine.dt))
        for j in range(per_seed):
            lead = leads[j % len(leads)]
            restrict(fine, ca)
            if lead > 0:
                learned_step(ca, net, lead)
                fine.step(lead * dt_factor)
                if ca.invariants()[2] != 0:      # the learned model diverged: no sample
                    fine.step(every - lead * dt_factor)
                    continue
            if gen is not None and j % 2 == 1:
                sig = torch.tensor([noise[0], noise[1], noise[2], noise[2]], device="cuda")
                dn = torch.randn((pc.n_theta, pc.n_phi, 4), generator=gen, device="cuda") * sig
                apply_correction(ca, dn.contiguous())
            ca.step(1)
            fine.step(dt_factor)
            restrict(fine, cb)
            learn_pair(ca, cb, m[i], y[i])
            fine.step(every - (lead + 1) * dt_factor)
            if reject is not None and lead > 0:
                _, s2 = learn_stats(y[i])
                rms = np.sqrt(s2 / (pc.n_theta * pc.n_phi))
                scale = np.asarray(reject[0], dtype=np.float64)
                if np.any((scale > 0) & (rms > reject[1] * scale)):
                    continue
            i += 1
        torch.cuda.synchronize()
        if progress:
            progress(f"pairs: seed {seed}: {per_seed} samples, {time.time() - t0:.1f} s")
        fine.close()
    return m[:i], y[:i]


def generate_shadow_pairs(p_fine, seeds, t_first, t_last, every, apply_mask=0, k=4,
                          dt_factor=4, precision=32, coarse_override=None, progress=print):
    """Training pairs from a coarse "shadow" run that follows each fine spinodal run: at
    t_first the fine state is restricted onto the coarse grid once; from then on the coarse
    grid takes its own steps and after each one is corrected by the exact target (restricted
    fine moments minus its own) in the channels of apply_mask (0 = all).  Its moments thus
    track the fine solution while its populations' non-equilibrium part -- a slow variable
    when the relaxation time spans many coarse steps -- evolves under the coarse dynamics, as
    it does under the learned step.  A sample is stored every `every` fine steps."""
    import torch
    assert every % dt_factor == 0
    pc = coarse_params(p_fine, k, dt_factor, **(coarse_override or {}))
    n_coarse = (_steps(t_last, p_fine.dt) - _steps(t_first, p_fine.dt)) // dt_factor
    per_seed = n_coarse // (every // dt_factor)
    shape = (len(seeds) * per_seed, pc.n_theta, pc.n_phi, 4)
    m = torch.empty(shape, dtype=torch.float32, device="cuda")
    y = torch.empty(shape, dtype=torch.float32, device="cuda")
    mt = torch.empty(shape[1:], dtype=torch.float32, device="cuda")
    yt = torch.empty(shape[1:], dtype=torch.float32, device="cuda")
    mask = torch.tensor([1.0 if (apply_mask == 0 or (apply_mask >> c) & 1) else 0.0
                         for c in range(4)], device="cuda")
    shadow, truth = TorusGrid(pc, precision), TorusGrid(pc, precision)
    i = 0
    for seed in seeds:
        t0 = time.time()
        fine = TorusGrid(p_fine, precision)
        fine.set_state(inputs.spinodal_phi(p_fine, seed=seed),
                       *inputs.rest_moments(p_fine.n_theta, p_fine.n_phi))
        fine.step(_steps(t_first, p_fine.dt))
        restrict(fine, shadow)
        for c in range(1, per_seed * (every // dt_factor) + 1):
            shadow.step(1)
            fine.step(dt_factor)
            restrict(fine, truth)
            sample = c % (every // dt_factor) == 0
            mm, yy = (m[i], y[i]) if sample else (mt, yt)
            learn_pair(shadow, truth, mm, yy)
            apply_correction(shadow, (yy * mask).contiguous())
            if sample:
                i += 1
        torch.cuda.synchronize()
        if progress:
            progress(f"shadow pairs: seed {seed}: {per_seed} samples, {time.time() - t0:.1f} s")
        fine.close()
    return m[:i], y[:i]


def normalisation(m, y):
    """Input shift/scale (mean and 1/std of each moment channel) and output scale (std of
    each target channel), from the data by the library's FP64 sums."""
    count = m.numel() // 4
    s, s2 = learn_stats(m)
    mean = s / count
    std = np.sqrt(np.maximum(s2 / count - mean * mean, 0.0))
    ts, ts2 = learn_stats(y)
    tstd = np.sqrt(np.maximum(ts2 / count - (ts / count) ** 2, 0.0))
    in_scale = 1.0 / np.maximum(std, 1e-12)
    out_scale = np.maximum(tstd, 1e-12)
    return dict(in_shift=mean, in_scale=in_scale, out_scale=out_scale)


def make_network(pc, norm, max_batch, seed, loss_weight=(1.0, 1.0, 1.0, 1.0), apply_mask=0):
    net = CoarseCNN(pc.r, pc.R, pc.n_theta, pc.n_phi, max_batch, norm["in_shift"],
                    norm["in_scale"], norm["out_scale"], loss_weight, apply_mask)
    net.set_params(inputs.cnn_init_params(seed))
    return net


def train(net, m, y, iters, batch, lr=2e-3, lr_final=5e-5, seed=0, report_every=200,
          progress=print):
    """Adam with a cosine learning-rate decay; batches drawn (seeded) from the samples.
    Returns the reported losses [(iteration, loss)]."""
    rng = np.random.default_rng(seed)
    n = m.shape[0]
    history = []
    t0 = time.time()
    for it in range(1, iters + 1):
        lr_it = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * (it - 1) / max(iters - 1, 1)))
        idx = rng.choice(n, size=min(batch, n), replace=False)
        want = it == 1 or it % report_every == 0 or it == iters
        loss = net.train_step(m, y, idx, it, lr_it, want_loss=want)
        if want:
            history.append((it, loss))
            if progress:
                progress(f"train: iter {it} loss {loss:.4e} lr {lr_it:.2e} ({time.time() - t0:.1f} s)")
    return history


def batch_loss(net, m, y, batch=16):
    """Mean loss of the network over all samples (weights unchanged), and of a zero
    correction (the plain coarse step) on the same samples."""
    n = m.shape[0]
    total, zero, cnt = 0.0, 0.0, 0
    w = np.array(net.desc.loss_weight[:4])
    s = np.array(net.desc.out_scale[:4])
    for b0 in range(0, n, batch):
        idx = list(range(b0, min(n, b0 + batch)))
        loss, _ = net.gradient(m, y, idx=idx)
        total += loss * len(idx)
        cnt += len(idx)
    ss, ss2 = learn_stats(y)
    zero = float(np.sum(w * ss2 / (s * s)) / (4 * (y.numel() // 4)))
    return total / cnt, zero


def _phi_l2(a, b):
    """Relative L2 difference of the phi fields of two grids of one shape."""
    pa = a.get_state()[1].double()
    pb = b.get_state()[1].double()
    return float(((pa - pb).norm() / pb.norm()).item())


def evaluate(p_fine, net, seed, t_start, t_end, every_t, k=4, dt_factor=4, precision=32,
             coarse_override=None, progress=print):
    """Hand the fine state at t_start over to a learned and a plain coarse grid and run all
    three to t_end; every every_t report the coarsening lengths L_d = A_total / L_I and L_S
    (structure factor) of the fine grid, of the restricted fine state on the coarse grid (the
    judge), of the learned and of the plain coarse grid, and the relative L2 difference of phi
    from the restricted fine state."""
    import torch
    pc = coarse_params(p_fine, k, dt_factor, **(coarse_override or {}))
    fine = TorusGrid(p_fine, precision)
    fine.set_state(inputs.spinodal_phi(p_fine, seed=seed),
                   *inputs.rest_moments(p_fine.n_theta, p_fine.n_phi))
    fine.step(_steps(t_start, p_fine.dt))
    judge, lc, pl = TorusGrid(pc, precision), coarse_grid(pc, precision), coarse_grid(pc, precision)
    restrict(fine, lc)
    restrict(fine, pl)
    rows = []
    n_chunks = _steps(t_end - t_start, every_t)
    fine_steps = _steps(every_t, p_fine.dt)
    coarse_steps = fine_steps // dt_factor
    assert coarse_steps * dt_factor == fine_steps
    for c in range(1, n_chunks + 1):
        fine.step(fine_steps)
        learned_step(lc, net, coarse_steps)
        pl.step(coarse_steps)
        restrict(fine, judge)
        L = [g.diagnostics(profiles=False)["L_d"] for g in (fine, judge, lc, pl)]
        S = [g.structure_length()[0] for g in (fine, judge, lc, pl)]
        row = dict(t=t_start + c * every_t, L_fine=L[0], L_judge=L[1], L_learned=L[2],
                   L_plain=L[3], LS_fine=S[0], LS_judge=S[1], LS_learned=S[2], LS_plain=S[3],
                   phi_l2_learned=_phi_l2(lc, judge), phi_l2_plain=_phi_l2(pl, judge),
                   nonfinite=lc.invariants()[2])
        rows.append(row)
        if progress:
            progress(f"eval t={row['t']:.1f}: L_d judge {L[1]:.4f} learned {(L[2] - L[1]) / L[1]:+.3f} "
                     f"plain {(L[3] - L[1]) / L[1]:+.3f} | L_S judge {S[1]:.4f} learned "
                     f"{(S[2] - S[1]) / S[1]:+.3f} plain {(S[3] - S[1]) / S[1]:+.3f} | phi L2 "
                     f"learned {row['phi_l2_learned']:.3f} plain {row['phi_l2_plain']:.3f}")
    torch.cuda.synchronize()
    return rows


def time_per_unit(p, stepper, steps, warmup=2):
    """Seconds of GPU time per unit of simulated time for `stepper(n)` on a grid of params p."""
    import torch
    stepper(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    stepper(steps)
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / (steps * p.dt)


class LearnedCoarseRunner:
    """The learned coarse step with the plain fine solver as judge and fallback.

    validate() runs the judged evaluation on a held-out seed and accepts the network only if
    the relative errors of L_S and L_d stay within max_error over the window; run() then advances a fine
    state handed over at some time by the learned coarse step, and falls back to the fine
    solver (from the handed-over state) if the network was not accepted or the coarse state
    turns non-finite."""

    def __init__(self, p_fine, net, k=4, dt_factor=4, max_error=0.02, precision=32,
                 coarse_override=None):
        self.p_fine, self.net, self.k, self.dt_factor = p_fine, net, k, dt_factor
        self.max_error, self.precision = max_error, precision
        self.coarse_override = coarse_override
        self.accepted = False
        self.report = None

    def validate(self, seed, t_start, t_end, every_t, progress=print):
        rows = evaluate(self.p_fine, self.net, seed, t_start, t_end, every_t, self.k,
                        self.dt_factor, self.precision, self.coarse_override, progress)
        # the larger of the L_S and L_d errors
        err = max(max(abs(r[k + "_learned"] - r[k + "_judge"]) / r[k + "_judge"]
                      for k in ("L", "LS")) for r in rows)
        err_plain = max(max(abs(r[k + "_plain"] - r[k + "_judge"]) / r[k + "_judge"]
                            for k in ("L", "LS")) for r in rows)
        self.accepted = err <= self.max_error and all(r["nonfinite"] == 0 for r in rows)
        self.report = dict(rows=rows, L_error=err, L_error_plain=err_plain,
                           accepted=self.accepted)
        return self.report

    def run(self, fine_grid, t_span):
        """Advance the state of fine_grid by t_span.  Returns ("learned", coarse grid) or
        ("fine", fine_grid) -- the latter after the fine solver has taken over."""
        pc = coarse_params(self.p_fine, self.k, self.dt_factor, **(self.coarse_override or {}))
        if self.accepted:
            coarse = coarse_grid(pc, self.precision)
            restrict(fine_grid, coarse)
            learned_step(coarse, self.net, _steps(t_span, pc.dt))
            if coarse.invariants()[2] == 0:
                return "learned", coarse
        fine_grid.step(_steps(t_span, self.p_fine.dt))
        return "fine", fine_grid
