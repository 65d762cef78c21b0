"""Train the learned coarse step for the spinodal coarsening workload and store its weights.

    python -m paper_1904_10070_amd.train_coarse [--tau 0.6] [--out DIR]

Recipe (all field work in libtlb's kernels, see learn.py):
  * fine grid 512 x 1280 (r = 1, R = 2.5, M = 2.5e-3, dt = 4e-4, interface width by the
    three-cell rule); coarse grid 128 x 320 with the same physical parameters and dt = 1.6e-3;
  * training pairs from shadow runs that follow fine runs of seeds 1, 2, 3, 5, 6 over
    t in [16, 44], a sample every 400 fine steps;
  * the network corrects phi and the velocity (apply mask 0b1101); loss weights
    (1, 0, 1/4, 1/4); Adam, 6000 iterations of 16 samples, cosine decay from 2e-3;
  * several initialisations are trained; the fine solver judges each on a held-out seed
    (hand-over at t = 20, L_d compared up to t = 32) and the one with the smallest largest
    L_d error is kept.
Writes <out>/learned_coarse_tau<tau>.bin (FP32 weights) and .json (normalisation, mask,
recipe and the judge's report).
"""
import argparse
import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS_DIR = os.path.join(HERE, "weights")

RECIPE = dict(train_seeds=(1, 2, 3, 5, 6), t_first=16.0, t_last=44.0, every=400,
              apply_mask=13, loss_weight=(1.0, 0.0, 0.25, 0.25), iters=6000, batch=16,
              lr=2e-3, init_seeds=(0, 1, 2), validate_seed=8, validate_t=(20.0, 32.0, 4.0))


def weights_path(tau, out=WEIGHTS_DIR):
    return os.path.join(out, f"learned_coarse_tau{tau:g}")


def load(tau, out=WEIGHTS_DIR):
    """(params float32[30660], metadata dict) of stored weights; raises if absent."""
    base = weights_path(tau, out)
    with open(base + ".json") as fh:
        meta = json.load(fh)
    params = np.fromfile(base + ".bin", dtype=np.float32)
    if params.size != meta["param_count"]:
        raise RuntimeError(f"{base}.bin holds {params.size} values, expected {meta['param_count']}")
    return params, meta


def network_from(meta, params, max_batch=1):
    from .binding import CoarseCNN
    g = meta["coarse"]
    net = CoarseCNN(g["r"], g["R"], g["n_theta"], g["n_phi"], max_batch, meta["in_shift"],
                    meta["in_scale"], meta["out_scale"], meta["loss_weight"], meta["apply_mask"])
    net.set_params(params)
    return net


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--tau", type=float, default=0.6)
    ap.add_argument("--out", default=WEIGHTS_DIR)
    ap.add_argument("--candidates", type=int, default=len(RECIPE["init_seeds"]))
    args = ap.parse_args(argv)

    import torch
    from . import inputs, learn as L

    R = RECIPE
    pf = inputs.spinodal_workload(args.tau)
    pc = L.coarse_params(pf)
    t0 = time.time()
    m, y = L.generate_shadow_pairs(pf, R["train_seeds"], R["t_first"], R["t_last"], R["every"],
                                   apply_mask=R["apply_mask"])
    t_data = time.time() - t0
    norm = L.normalisation(m, y)
    best = None
    for init in R["init_seeds"][:args.candidates]:
        t1 = time.time()
        net = L.make_network(pc, norm, R["batch"], seed=init, loss_weight=R["loss_weight"],
                             apply_mask=R["apply_mask"])
        hist = L.train(net, m, y, R["iters"], R["batch"], lr=R["lr"], seed=init,
                       report_every=R["iters"] // 4)
        torch.cuda.synchronize()
        t_train = time.time() - t1
        vs, ve, vk = R["validate_t"]
        rows = L.evaluate(pf, net, R["validate_seed"], vs, ve, vk)
        errs = [abs(r["L_learned"] - r["L_judge"]) / r["L_judge"] for r in rows]
        err = max(errs) if all(np.isfinite(errs)) else float("inf")
        print(f"candidate {init}: largest L_d error on seed {R['validate_seed']} over "
              f"t in [{vs}, {ve}]: {err:.4f} (training {t_train:.1f} s)", flush=True)
        if best is None or err < best[0]:
            best = (err, init, net.get_params(), rows, hist, t_train)
        net.close()
    err, init, params, rows, hist, t_train = best
    os.makedirs(args.out, exist_ok=True)
    base = weights_path(args.tau, args.out)
    params.astype(np.float32).tofile(base + ".bin")
    meta = dict(tau=args.tau, param_count=int(params.size),
                coarse=dict(r=pc.r, R=pc.R, n_theta=pc.n_theta, n_phi=pc.n_phi, dt=pc.dt),
                fine=dict(n_theta=pf.n_theta, n_phi=pf.n_phi, dt=pf.dt, kappa=pf.kappa, A=pf.A,
                          M=pf.M, tau=pf.tau),
                in_shift=[float(v) for v in norm["in_shift"]],
                in_scale=[float(v) for v in norm["in_scale"]],
                out_scale=[float(v) for v in norm["out_scale"]],
                loss_weight=list(R["loss_weight"]), apply_mask=R["apply_mask"],
                recipe={k: (list(v) if isinstance(v, tuple) else v) for k, v in R.items()},
                chosen_init=init, samples=int(m.shape[0]), data_seconds=round(t_data, 1),
                train_seconds=round(t_train, 1),
                loss_history=[[int(i), float(l)] for i, l in hist],
                validation=dict(seed=R["validate_seed"], largest_L_error=err, rows=rows))
    with open(base + ".json", "w") as fh:
        json.dump(meta, fh, indent=1)
    print(f"kept candidate {init} (largest L_d error {err:.4f}); wrote {base}.bin/.json", flush=True)


if __name__ == "__main__":
    main()
