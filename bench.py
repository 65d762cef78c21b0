"""Throughput of the torus step on one MI355X: node-updates per second and HBM roofline.

A step is one full time step of the method (three fused stage launches of the SSP-RK3
integrator: moments, chemical potential, interface force, BGK, upwind advection, velocity-space
force and connection terms, Cahn-Hilliard) over the whole grid, with the state resident in HBM.

Headline workload: spinodal coarsening on a 512 x 1280 torus (r = 1, R = 2.5, tau = 0.6,
M = 2.5e-3, phi ~ U[-0.1, 0.1] from seed 7, n = 1, u = 0), populations stored and stepped in
FP32.  The same line also carries the FP64 rate on that workload, the FP32 rate on a
2048 x 5120 grid whose working set (2.1 GB) is far larger than the 256 MB last-level cache, the
batched ensemble of 64 tori against separate runs, and the learned coarse step's speedup over
the fine FP32 step with its coarsening-length errors against the fine solver.

Roofline: the stage kernel is HBM-bound.  Algorithmic traffic per node and time step is 136
values (stage 1 reads y^n and writes y1: 16 + 16 populations, 1 + 1 phi; stages 2 and 3 read
y_s and y^n and write one copy: 32 + 16 populations and 2 + 1 phi each), i.e. 544 B in FP32 and
1088 B in FP64.  `achieved` is those bytes per launch (one third of a step) over the average
launch time, measured with HIP events on the stream the kernels run on.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALUES_PER_NODE_STEP = 136
REPS = 5            # timed repetitions of every measurement; the median is reported
GRAPH_CHUNK = 32    # the library replays graphs of 32 time steps


def algorithmic_bytes_per_node_step(precision):
    return VALUES_PER_NODE_STEP * (4 if precision == 32 else 8)


def spread(ts):
    """median, min, max and (max - min) / median of a list of times."""
    xs = sorted(ts)
    med = xs[len(xs) // 2] if len(xs) % 2 else 0.5 * (xs[len(xs) // 2 - 1] + xs[len(xs) // 2])
    return dict(median=med, min=xs[0], max=xs[-1], spread=(xs[-1] - xs[0]) / med)


def event_reps(run, stream, reps=REPS):
    """Seconds of each of `reps` calls of run(), timed with HIP events recorded on `stream`
    (the stream the kernels are launched on), with a synchronisation on both sides."""
    import torch
    out = []
    for _ in range(reps):
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        run()
        stop.record(stream)
        torch.cuda.synchronize()
        out.append(start.elapsed_time(stop) * 1e-3)
    return out


def graph_steps(t_step, seconds):
    """A step count for a timed repetition of about `seconds`: a multiple of the graph chunk,
    at least two chunks, so that every step is a graph replay."""
    n = max(2 * GRAPH_CHUNK, int(seconds / max(t_step, 1e-9)))
    return (n + GRAPH_CHUNK - 1) // GRAPH_CHUNK * GRAPH_CHUNK


def new_grid(p, precision, seed=7, phi=None):
    from paper_1904_10070_amd import TorusGrid, inputs
    g = TorusGrid(p, precision=precision)
    phi = inputs.spinodal_phi(p, seed=seed) if phi is None else phi
    g.set_state(phi, *inputs.rest_moments(p.n_theta, p.n_phi))
    return g


def leg_result(p, precision, ts_per_step, steps):
    """node-updates/s and the roofline figures of a median time per step."""
    st = spread(ts_per_step)
    t_step = st["median"]
    nodes = p.n_theta * p.n_phi
    bytes_launch = algorithmic_bytes_per_node_step(precision) * nodes / 3.0
    achieved = bytes_launch / (t_step / 3.0) / 1e9
    return dict(nups=nodes / t_step, t_step=t_step, achieved_gbs=achieved,
                bytes_per_launch=bytes_launch, steps=steps,
                timing={"reps": len(ts_per_step), "steps_per_rep": steps,
                        "ms_per_step_median": t_step * 1e3, "ms_per_step_min": st["min"] * 1e3,
                        "ms_per_step_max": st["max"] * 1e3, "spread": st["spread"]})


def gpu_busy(seconds=0.15, mib=1024):
    """About `seconds` of the project's copy kernel on a scratch buffer: brings the GPU to its
    steady clocks right before a short timed region, without stepping any grid."""
    import torch
    from paper_1904_10070_amd.binding import hbm_stream, STREAM_COPY
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    z = torch.empty(n, dtype=torch.float32, device="cuda")
    calls = max(1, int(seconds / (2 * mib * (1 << 20) / 6.0e12)))
    for _ in range(calls):
        hbm_stream(STREAM_COPY, x, None, z)
    torch.cuda.synchronize()
    del x, z


def gpu_leg(p, precision, steps, warmup, seed=7, phi=None, rows=None):
    """`warmup` untimed steps, then REPS timed repetitions of exactly `steps` steps, after a
    fraction of a second of other GPU work (a few warm-up steps leave the clocks below their
    steady state: 20-step blocks right after 5 warm-up steps measured 10-15 % slower than the
    same blocks later in the same process)."""
    g = new_grid(p, precision, seed, phi)
    if rows:
        g.set_tile_rows(rows)
    g.step(warmup)
    gpu_busy()
    ts = [t / steps for t in event_reps(lambda: g.step(steps), g.stream)]
    bad = g.invariants()[2]
    g.close()
    return dict(leg_result(p, precision, ts, steps), nonfinite=bad)


def graph_leg(p, precision, seconds=1.0, seed=7, phi=None, grid=None):
    """REPS repetitions of about `seconds` each, every step a graph replay (two warm-up chunks
    build the graph first)."""
    g = grid if grid is not None else new_grid(p, precision, seed, phi)
    g.step(2 * GRAPH_CHUNK)
    probe = event_reps(lambda: g.step(2 * GRAPH_CHUNK), g.stream, reps=1)[0] / (2 * GRAPH_CHUNK)
    steps = graph_steps(probe, seconds)
    ts = [t / steps for t in event_reps(lambda: g.step(steps), g.stream)]
    bad = g.invariants()[2]
    if grid is None:
        g.close()
    return dict(leg_result(p, precision, ts, steps), nonfinite=bad)


def leg_json(d, **extra):
    return dict({"value": d["nups"], "unit": "node-updates/s", "ms_per_step": d["t_step"] * 1e3,
                 "steps": d["steps"], "roofline_frac": d["achieved_gbs"] / HBM_PEAK_GBS,
                 "achieved_gbs": d["achieved_gbs"], "timing": d["timing"]}, **extra)


def ensemble_leg(seconds=0.5):
    """64 tori (inputs.ensemble_workload) in FP32: one fused launch per stage for the whole
    ensemble (autotuned tile height) against the same grids stepped one after another, both
    graph-replayed (step counts a multiple of the 32-step chunk), REPS repetitions each."""
    from paper_1904_10070_amd import TorusBatch, TorusGrid, inputs
    params = inputs.ensemble_workload()
    grids = []
    for i, p in enumerate(params):
        g = TorusGrid(p, precision=32)
        g.set_state(inputs.spinodal_phi(p, seed=1000 + i), *inputs.rest_moments(p.n_theta, p.n_phi))
        grids.append(g)
    nodes = sum(p.n_theta * p.n_phi for p in params)
    batch = TorusBatch(grids)
    rows = batch.autotune()
    stream = grids[0].stream
    batch.step(2 * GRAPH_CHUNK)
    probe = event_reps(lambda: batch.step(2 * GRAPH_CHUNK), stream, reps=1)[0] / (2 * GRAPH_CHUNK)
    steps = graph_steps(probe, seconds)
    tb = spread([t / steps for t in event_reps(lambda: batch.step(steps), stream)])

    def alone():
        for g in grids:
            g.step(steps)
    alone_warm = [g.step(2 * GRAPH_CHUNK) for g in grids]
    del alone_warm
    ta = spread([t / steps for t in event_reps(alone, stream)])
    batch.close()
    for g in grids:
        g.close()
    t_batch, t_alone = tb["median"], ta["median"]
    achieved = 544.0 * nodes / t_batch / 1e9
    return {"value": nodes / t_batch, "unit": "node-updates/s", "tori": len(params),
            "nodes": nodes, "ms_per_step": t_batch * 1e3, "tile_rows": rows,
            "state_bytes": 51 * 4 * nodes, "streaming": 51 * 4 * nodes > (1 << 30),
            "roofline_frac": achieved / HBM_PEAK_GBS, "achieved_gbs": achieved,
            "separate_runs_value": nodes / t_alone, "speedup_vs_separate": t_alone / t_batch,
            "steps": steps, "graph_replayed": True,
            "timing": {"reps": REPS, "batch_spread": tb["spread"], "separate_spread": ta["spread"]}}


def learned_leg(t_fine_step, steps=2048, seeds=(7, 9, 10), t_start=20.0, t_end=30.0,
                every_t=2.0):
    """The learned coarse step (128 x 320, 4x time step, weights trained by train_coarse.py)
    on held-out seeds: for each, the fine FP32 solver runs the spinodal workload to t_start,
    hands its state to a learned and a plain coarse grid, and judges both up to t_end by the
    coarsening lengths of the restricted fine state (structure-factor L_S and
    L_d = A_total / L_I); the largest errors over the seeds are reported.  Speed: GPU time per
    unit of simulated time of the learned and plain coarse steps (graph-replayed) against the
    fine FP32 step (graph-replayed, `t_fine_step`)."""
    from paper_1904_10070_amd import inputs, learn as L, train_coarse
    from paper_1904_10070_amd.binding import learned_step
    params, meta = train_coarse.load(0.6)
    net = train_coarse.network_from(meta, params)
    pf = inputs.spinodal_workload(0.6)
    pc = L.coarse_params(pf)
    per_seed = {}
    rows7 = None
    for seed in seeds:
        rows = L.evaluate(pf, net, seed, t_start, t_end, every_t, progress=None)
        if rows7 is None:
            rows7 = rows
        rel = lambda a, b: [abs(r[a] - r[b]) / r[b] for r in rows]  # noqa: E731
        per_seed[str(seed)] = {"L_S_error_max": max(rel("LS_learned", "LS_judge")),
                               "L_d_error_max": max(rel("L_learned", "L_judge")),
                               "L_S_error_max_plain_coarse": max(rel("LS_plain", "LS_judge")),
                               "L_d_error_max_plain_coarse": max(rel("L_plain", "L_judge")),
                               "phi_l2_end": rows[-1]["phi_l2_learned"],
                               "phi_l2_end_plain_coarse": rows[-1]["phi_l2_plain"]}

    def per_step(stepper):
        g = L.coarse_grid(pc, precision=32)
        g.set_state(inputs.spinodal_phi(pc, seed=seeds[0]), *inputs.rest_moments(pc.n_theta, pc.n_phi))
        stepper(g, 2 * GRAPH_CHUNK)
        ts = [t / steps for t in event_reps(lambda: stepper(g, steps), g.stream)]
        g.close()
        return spread(ts)["median"]

    t_learned = per_step(lambda g, n: learned_step(g, net, n))
    t_plain = per_step(lambda g, n: g.step(n))
    fine_per_t = t_fine_step / pf.dt
    worst = lambda k: max(v[k] for v in per_seed.values())  # noqa: E731
    return {"workload": f"spinodal {pf.n_theta}x{pf.n_phi} (tau=0.6) -> learned coarse "
                        f"{pc.n_theta}x{pc.n_phi}, dt x{round(pc.dt / pf.dt)}; hand-over at "
                        f"t={t_start:g} from held-out seeds {list(seeds)}, judged to t={t_end:g}",
            "L_S_error_max": worst("L_S_error_max"), "L_d_error_max": worst("L_d_error_max"),
            "L_S_error_max_plain_coarse": worst("L_S_error_max_plain_coarse"),
            "L_d_error_max_plain_coarse": worst("L_d_error_max_plain_coarse"),
            "per_seed": per_seed,
            "speedup_vs_fine_fp32": fine_per_t / (t_learned / pc.dt),
            "speedup_plain_coarse": fine_per_t / (t_plain / pc.dt),
            "ms_per_learned_step": t_learned * 1e3, "ms_per_plain_coarse_step": t_plain * 1e3,
            "ms_per_fine_step": t_fine_step * 1e3, "steps_timed": steps, "graph_replayed": True,
            "rows_seed_%d" % seeds[0]: [{k: (round(v, 5) if isinstance(v, float) else v)
                                        for k, v in r.items()} for r in rows7],
            "training_record": {"note": "copied from the weights' metadata (written by "
                                        "train_coarse.py when the weights were trained); not "
                                        "measured in this run",
                                "samples": meta["samples"], "data_s": meta["data_seconds"],
                                "train_s": meta["train_seconds"],
                                "validation_seed": meta["validation"]["seed"],
                                "validation_L_error": meta["validation"]["largest_L_error"]}}


def learned_step_timing(steps=2048):
    """GPU time per learned and per plain coarse step on the 128 x 320 grid (profiling runs)."""
    from paper_1904_10070_amd import inputs, learn as L, train_coarse
    from paper_1904_10070_amd.binding import learned_step
    params, meta = train_coarse.load(0.6)
    net = train_coarse.network_from(meta, params)
    pc = L.coarse_params(inputs.spinodal_workload(0.6))
    out = {}
    for name, stepper in (("learned", lambda g, n: learned_step(g, net, n)),
                          ("plain", lambda g, n: g.step(n))):
        g = L.coarse_grid(pc, precision=32)
        out[f"tile_rows_{name}"] = g.tile_rows
        g.set_state(inputs.spinodal_phi(pc, seed=7), *inputs.rest_moments(pc.n_theta, pc.n_phi))
        stepper(g, 2 * GRAPH_CHUNK)
        ts = [t / steps for t in event_reps(lambda: stepper(g, steps), g.stream)]
        out[f"ms_per_{name}_step"] = spread(ts)["median"] * 1e3
        g.close()
    return out


# algorithmic multiply-add work of the network per node: sum over layers of 2 * 9 * c_in * c_out
# (forward), the same again for the weight gradient, and for the input gradient of layers 1..4
CNN_ARCH = ((6, 32), (32, 32), (32, 32), (32, 32), (32, 4))
CNN_FWD_FLOP = sum(2 * 9 * ci * co for ci, co in CNN_ARCH)
CNN_TRAIN_FLOP = 2 * CNN_FWD_FLOP + sum(2 * 9 * ci * co for ci, co in CNN_ARCH[1:])


def training_timing(iters=200, batch=16):
    """Training steps of the network on seeded synthetic pairs of the 128 x 320 coarse grid:
    time per step and the algorithmic bf16 matrix-core rate it implies."""
    import torch
    from paper_1904_10070_amd import inputs
    from paper_1904_10070_amd.binding import CoarseCNN
    H, W, S = 128, 320, 64
    m, y = inputs.learn_samples(3, S, H, W)
    m, y = torch.tensor(m, device="cuda"), torch.tensor(y, device="cuda")
    net = CoarseCNN(1.0, 2.5, H, W, batch, (0.0, 1.0, 0.0, 0.0), (1.0, 50.0, 100.0, 100.0),
                    (1e-3, 1e-6, 1e-5, 1e-5))
    net.set_params(inputs.cnn_init_params(0))
    rng = __import__("numpy").random.default_rng(0)
    idx = [rng.choice(S, size=batch, replace=False) for _ in range(iters + 10)]
    for it in range(10):
        net.train_step(m, y, idx[it], it + 1, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(iters):
        net.train_step(m, y, idx[10 + it], 11 + it, 1e-4)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / iters
    flop = CNN_TRAIN_FLOP * batch * H * W
    return {"ms_per_train_step": dt * 1e3, "batch": batch, "grid": f"{H}x{W}",
            "tflops": flop / dt / 1e12, "bf16_peak_tflops": 2500.0,
            "frac": flop / dt / 1e12 / 2500.0}


def measured_traffic(key):
    """HBM bytes per launch of the stage kernel from the committed counter summary
    (profiles/stage_kernel_traffic.json), or None if the kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "stage_kernel_traffic.json")
    src = os.path.join(ROOT, "paper_1904_10070_amd", "csrc", "tlb.hip")
    try:
        rec = json.load(open(path))
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != digest:
        return None
    return rec.get("traffic_bytes_per_launch", {}).get(key)


def stream_ceiling(gib=2.0, reps=20):
    """The project's HBM streaming kernels (tlb_hbm_stream) on buffers of `gib` GiB each:
    copy (1 read : 1 write), add (2 : 1) and read-only rates, median of `reps` calls after one
    untimed call, each timed with HIP events on the current stream.  `stage_mix_gbs` is the
    rate of the stage kernel's traffic mix at these rates: stage 1 moves 34 values at 1 : 1 and
    stages 2 and 3 51 values each at 2 : 1 per node and step."""
    import torch
    from paper_1904_10070_amd.binding import hbm_stream, STREAM_COPY, STREAM_ADD, STREAM_READ
    n = int(gib * (1 << 30)) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.ones(n, dtype=torch.float32, device="cuda")
    z = torch.empty(n, dtype=torch.float32, device="cuda")
    parts = torch.empty(4 * 8192, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    out = {}
    for name, mode, a, b, c in (("copy", STREAM_COPY, x, None, z), ("add", STREAM_ADD, x, y, z),
                                ("read", STREAM_READ, x, None, parts)):
        moved = hbm_stream(mode, a, b, c)
        ts = event_reps(lambda: hbm_stream(mode, a, b, c), stream, reps=reps)
        out[name + "_gbs"] = moved / spread(ts)["median"] / 1e9
    del x, y, z
    torch.cuda.empty_cache()
    t_mix = 34.0 / out["copy_gbs"] + 2 * 51.0 / out["add_gbs"]
    out["stage_mix_gbs"] = (34.0 + 2 * 51.0) / t_mix
    out["buffer_gib"] = gib
    out["kernel"] = "tlb_stream_kernel (include/tlb_stream.h), 16 B per lane, nontemporal"
    return out


def copy_bandwidth(mib=1024, reps=20):
    """Read+write bandwidth of a plain device-to-device copy (torch) of `mib` MiB, for context
    next to the project's own streaming kernels."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ts = event_reps(lambda: dst.copy_(src), torch.cuda.current_stream(), reps=reps)
    return 8.0 * n / spread(ts)["median"] / 1e9


CPU_SCRIPT = """
import json, os, sys, time
sys.path.insert(0, sys.argv[1])
from oracle import ref
from paper_1904_10070_amd import inputs
p = inputs.drop_workload()
g = ref.RefGrid(**p.as_dict())
g.set_state(inputs.drop_workload_phi(p, seed=1), *inputs.rest_moments(p.n_theta, p.n_phi))
t0 = time.perf_counter()
g.step(2000)
dt = time.perf_counter() - t0
print(json.dumps({"value": p.n_theta * p.n_phi * 2000 / dt, "steps": 2000, "seconds": dt,
                  "threads": int(os.environ.get("OMP_NUM_THREADS", "0"))}))
"""


def cpu_config1(threads):
    """The FP64 oracle on the whole 64 x 160 drop workload (2000 steps), in a CPU-only child
    process with OMP_NUM_THREADS = threads (the thread count is fixed when the oracle loads)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS=str(threads), HIP_VISIBLE_DEVICES="")
    try:
        r = subprocess.run([sys.executable, "-c", CPU_SCRIPT, ROOT], env=env,
                           capture_output=True, text=True, timeout=300)
        return dict(json.loads(r.stdout.strip().splitlines()[-1]), unit="node-updates/s",
                    cores=threads, workload="drop 64x160 FP64, 2000 steps (whole workload)")
    except (subprocess.SubprocessError, ValueError, IndexError) as e:
        return {"error": str(e)[:200], "cores": threads}


def host_threads():
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def cpu_baseline(p, budget_s=12.0):
    """The FP64 oracle on the host cores: a bounded sample of the headline workload (a number
    of steps of about budget_s seconds after one warm-up step), plus the whole 64 x 160 drop
    workload on all threads and on one."""
    from oracle import ref
    from paper_1904_10070_amd import inputs
    g = ref.RefGrid(**p.as_dict())
    g.set_state(inputs.spinodal_phi(p, seed=7), *inputs.rest_moments(p.n_theta, p.n_phi))
    t0 = time.perf_counter()
    g.step(1)
    one = time.perf_counter() - t0
    n_more = max(1, min(50, int(budget_s / max(one, 1e-6)) - 1))
    t0 = time.perf_counter()
    g.step(n_more)
    dt = time.perf_counter() - t0
    g.close()
    threads = host_threads()
    return dict(value=p.n_theta * p.n_phi * n_more / dt, unit="node-updates/s", cores=threads,
                kind="oracle",
                sample=f"FP64 oracle, {n_more} steps of the {p.n_theta}x{p.n_phi} spinodal "
                       f"workload after 1 warm-up step ({dt:.1f} s), {threads} threads",
                config1_all_threads=cpu_config1(threads), config1_one_thread=cpu_config1(1))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="only the headline FP32 leg")
    ap.add_argument("--only", choices=["spinodal32", "spinodal64", "roofline32", "roofline64",
                                       "ensemble32", "learned32", "learnedstep32", "train32",
                                       "weno32", "stream"],
                    help="time a single workload/precision (profiling runs)")
    ap.add_argument("--rows", type=int, choices=[4, 8, 16],
                    help="tile height of the stage kernel for --only legs (default: the "
                         "library's 8)")
    ap.add_argument("--copy-calibration", type=int, metavar="MIB",
                    help="run only the project's copy kernel on MIB mebibytes, 20 times (the "
                         "reference kernel for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the torus step is measured on a single MI355X "
              "(multi-GPU sharding is designed but not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1904_10070_amd import inputs, load_library, WENO5, CH4
    load_library()
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    if args.copy_calibration:
        from paper_1904_10070_amd.binding import hbm_stream, STREAM_COPY
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        ts = event_reps(lambda: hbm_stream(STREAM_COPY, src, None, dst),
                        torch.cuda.current_stream(), reps=20)
        print(json.dumps({"copy_mib": args.copy_calibration, "bytes_read": 4 * n,
                          "bytes_written": 4 * n,
                          "gbs_read_plus_write": 8 * n / spread(ts)["median"] / 1e9}))
        return
    if args.only == "stream":
        print(json.dumps(stream_ceiling()))
        return
    if args.only == "ensemble32":
        print(json.dumps(ensemble_leg()))
        return
    if args.only == "learnedstep32":
        print(json.dumps(learned_step_timing(args.steps)))
        return
    if args.only == "train32":
        print(json.dumps(training_timing(args.steps)))
        return
    if args.only == "learned32":
        d = graph_leg(inputs.spinodal_workload(0.6), 32)
        print(json.dumps(learned_leg(d["t_step"])))
        return
    if args.only:
        wl, prec = args.only[:-2], int(args.only[-2:])
        p = inputs.spinodal_workload(0.6) if wl in ("spinodal", "weno") else inputs.roofline_workload()
        if wl == "weno":
            p = p.with_(flags=WENO5)
        d = gpu_leg(p, prec, args.steps, args.warmup, rows=args.rows)
        print(json.dumps({"workload": f"{wl} {p.n_theta}x{p.n_phi}", "precision": prec,
                          "rows": args.rows or 8,
                          "value": d["nups"], "unit": "node-updates/s",
                          "ms_per_step": d["t_step"] * 1e3, "achieved_gbs": d["achieved_gbs"],
                          "roofline_frac": d["achieved_gbs"] / HBM_PEAK_GBS,
                          "bytes_per_launch": d["bytes_per_launch"], "steps": args.steps,
                          "timing": d["timing"]}))
        return

    p = inputs.spinodal_workload(0.6)
    ceiling = stream_ceiling()
    head = gpu_leg(p, 32, args.steps, args.warmup)
    out = {
        "metric": "node-updates/s & % HBM peak, FP32 vs FP64; batched + learned-coarse speedup at err",
        "value": head["nups"],
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["t_step"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded spinodal initial condition, eq. phirand)",
        "config": {"workload": "spinodal coarsening torus 512x1280, r=1, R=2.5, tau=0.6, "
                               "M=2.5e-3, dt=4e-4, FP32 populations",
                   "n_theta": p.n_theta, "n_phi": p.n_phi, "parallelism": "single GPU"},
        "timing": dict(head["timing"], graph_replayed=True,
                       note="REPS repetitions of exactly `steps` steps after `warmup` steps and "
                            "0.15 s of copy-kernel work on a scratch buffer (clock warm-up); "
                            "value from the median. With few steps this times the start of the "
                            "run (random phi), which runs slower than the coarsened states "
                            "later on: fp32_graph_1s is the long-run rate"),
        "roofline": {"bound": "hbm", "achieved": head["achieved_gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": head["achieved_gbs"] / HBM_PEAK_GBS,
                     "traffic": measured_traffic("spinodal512x1280_fp32"),
                     "kernel": "tlb_stage_kernel<float>",
                     "bytes_per_launch": head["bytes_per_launch"],
                     "copy_gbs": ceiling["copy_gbs"], "stream": ceiling,
                     "frac_of_stream_mix": head["achieved_gbs"] / ceiling["stage_mix_gbs"],
                     "copy_gbs_torch": copy_bandwidth(),
                     # the same copy between two buffers of half the three state copies
                     # each (134 MB in all, which stays in the 256 MB last-level cache, as
                     # the working set of this grid does)
                     "copy_gbs_working_set_torch": copy_bandwidth(
                         mib=max(1, int(51 * p.n_theta * p.n_phi * 4 / 2 / (1 << 20))), reps=50)},
    }
    if not args.no_extra:
        d = graph_leg(p, 32, seconds=1.0)
        out["fp32_graph_1s"] = leg_json(d)
        t_fine = d["t_step"]
        d = graph_leg(p, 64, seconds=1.0)
        out["fp64"] = leg_json(d, traffic=measured_traffic("spinodal512x1280_fp64"))
        pr = inputs.roofline_workload()
        d = graph_leg(pr, 32, seconds=1.0)
        out["fp32_2048x5120"] = leg_json(
            d, frac_of_stream_mix=d["achieved_gbs"] / ceiling["stage_mix_gbs"],
            traffic=measured_traffic("roofline2048x5120_fp32"))
        # the small drop workload (64 x 160, FP64): launch-bound, stepped through the graph
        pd = inputs.drop_workload()
        d = graph_leg(pd, 64, seconds=0.25, phi=inputs.drop_workload_phi(pd, seed=1))
        out["drop64x160_fp64"] = leg_json(d)
        # the WENO-5 advection variant (nonlinear face weights: arithmetic-bound)
        d = graph_leg(p.with_(flags=WENO5), 32, seconds=0.5)
        out["weno5_fp32"] = leg_json(d, vs_uw5=d["nups"] / out["fp32_graph_1s"]["value"])
        # the fourth-order Cahn-Hilliard variant: a prepass per stage (reads the 16 populations
        # and phi, writes mu and the two advection fluxes) whose three planes the stage kernel
        # reads as halo tiles: 136 + 3 x 23 = 205 values per node and step.  Its surface
        # Laplacian has a larger spectral radius (the five-point fourth-order symbol reaches
        # 16/3 against 4), so the time step is halved to stay inside the explicit bound.
        d = graph_leg(p.with_(flags=CH4, dt=p.dt / 2), 32, seconds=0.5)
        ch4_gbs = 205 * 4 * d["nups"] / 1e9
        out["ch4_fp32"] = leg_json(d, vs_uw5=d["nups"] / out["fp32_graph_1s"]["value"],
                                   values_per_node_step=205, achieved_gbs_with_prepass=ch4_gbs,
                                   roofline_frac_with_prepass=ch4_gbs / HBM_PEAK_GBS,
                                   dt=p.dt / 2, nonfinite=d["nonfinite"])
        out["ensemble64_fp32"] = ensemble_leg()
        out["learned_coarse_fp32"] = learned_leg(t_fine)
        # the network's training step (16 samples of 128 x 320, bf16 matrix cores), measured
        out["cnn_training_bf16"] = training_timing(200)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
