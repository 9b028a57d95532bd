#!/usr/bin/env python3
"""Benchmark of the QCT hot path on one MI355X.

One step = one pass of the whole path over the full sweep of H2 + Ca
collisions (7744 instances: 64 log-spaced collision energies 1e2..1e5 K x
v 0..10 x j 0..10, 1292 trajectories each, b uniform in area to 12 a0;
10,005,248 trajectories): instance set-up with Bohr-Sommerfeld levels,
initial conditions, adaptive Runge-Kutta propagation (Dormand-Prince 8(5,3),
or the paper's 5(4)) of every trajectory to its stop rule in one persistent
launch, classification and Gaussian binning, per-instance cross sections and
rates.  All inputs are synthetic and seeded; nothing is cached between
steps.  Other workloads (--workload) are the 1e5-trajectory batched set, the
mixed-potential set, the paper's fixed-b grid and the 500-trajectory case.

Prints one JSON line: the metric, the roofline of the propagation kernel
(hand-counted FP64 work from the kernel source, with the method-only count
and the hardware-counter count beside it), the learned-proposal efficiency
(variance x GPU-seconds, plain / learned, with its 95 % interval), the
outcome counts by stop status, and the CPU oracle's baseline on a bounded
sample (a process pool on every host core, and one core).
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# FP64 operations per trial step of one trajectory, counted by hand from the
# step function's source (add, subtract, multiply 1; FMA 2; the hardware
# reciprocal and inverse-square-root estimates 1; rounding, scaling by 2^n,
# min/max/abs, compares and selects 0), per surface and RK variant:
#   hand    every operation the source performs, the software exponential
#           (Cody-Waite reduction and degree-11 polynomial, 27 FLOP) and the
#           Goldschmidt / Newton refinements of the square root (15 FLOP)
#           and reciprocal (5 FLOP) included;
#   method  the same with each exponential, square root and reciprocal
#           counted as one operation;
#   counter the hardware FP64 counters (64 (ADD + MUL + TRANS + 2 FMA) per
#           lane-step) of a full-wave fixed-step run of the one-lane kernel.
F_STEP = {("morse", 0): {"hand": 1886.0, "method": 1068.0, "counter": 1869.7},
          ("morse", 1): {"hand": 4072.0, "method": 2498.0, "counter": 4068.7},
          ("mixed", 0): {"hand": 1778.0, "method": 1128.0, "counter": 1743.6},
          ("mixed", 1): {"hand": 3856.0, "method": 2618.0, "counter": 3816.6}}
# HBM bytes per launch of the persistent kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes, scaled by the same counters on a plain copy of known
# size (bench.py --probe copy), keyed by (workload, kernel); a kernel changed
# since its counters were taken has no entry (null in the line).
TRAFFIC = {("h2ca_sweep_7744inst_1e7", "k_persistent<1,0,0,0,1>"): 5.673e9,
           ("h2ca_batched_96inst_1e5", "k_persistent<4,0,0,0,1>"): 3.242e7,
           ("mixed_2112inst_1e6", "k_persistent<1,3,0,2,1>"): 5.748e8,
           ("h2ca_paper_grid_v1j0", "k_persistent<1,0,0,0,1>"): 7.541e8}
RK_NAMES = {"dopri5": 0, "dop853": 1}
KINDS = {"morse": "0,0,0", "mixed": "3,0,2"}   # 3: LJ 12-6 specialisation
# workload -> (surface, CPU-baseline stride of the process pool, of one core)
WORKLOADS = {"sweep": ("morse", 1000, 10000), "batched": ("morse", 2, 50),
             "small": ("morse", 1, 5), "mixed": ("mixed", 500, 5000),
             "paper_grid": ("morse", 500, 5000)}
PEAK_FP64_VECTOR = 78.6e12   # MI355X, FLOP/s
STATUS_NAMES = ("running", "ok_rstop", "ok_tmax", "fail_maxsteps", "fail_nonfinite",
                "fail_hmin", "collapse")
LABEL_NAMES = ("quench", "r1", "r2", "diss", "unresolved", "failed")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sweep", choices=list(WORKLOADS))
    ap.add_argument("--cpu-stride", type=int, default=0,
                    help="CPU baseline pool runs every k-th trajectory id through the oracle "
                         "(0: the workload's default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-procs", type=int, default=16,
                    help="processes of the CPU baseline pool (the host's share of cores)")
    ap.add_argument("--rk", default="dop853", choices=list(RK_NAMES),
                    help="Runge-Kutta variant of the adaptive integrator")
    ap.add_argument("--atol", type=float, default=None, help="override the workload's atol")
    ap.add_argument("--rtol", type=float, default=None, help="override the workload's rtol")
    ap.add_argument("--path", default="run", choices=["run", "unfused"],
                    help="run: fused persistent launch (qcams_run); unfused: the four ABI calls")
    ap.add_argument("--autotune", action="store_true",
                    help="pick run options with qcams_autotune before timing")
    ap.add_argument("--blocks", type=int, default=0)
    ap.add_argument("--refill-min", type=int, default=1)
    ap.add_argument("--check-every", type=int, default=8)
    ap.add_argument("--no-lpt", action="store_true")
    ap.add_argument("--lanes", type=int, default=0, choices=[0, 1, 4, 8],
                    help="lanes per trajectory in the persistent kernel (0: by run size)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-proposal comparison (variance x GPU-seconds, learned "
                         "vs plain, dissociation of H2(v=4,j=0)+Ca at 5e4 K)")
    ap.add_argument("--learned-replicates", type=int, default=96)
    ap.add_argument("--learned-n", type=int, default=200_000)
    ap.add_argument("--learned-epochs", type=int, default=20)
    ap.add_argument("--probe", default="none", choices=["none", "flops", "copy", "mlp"],
                    help="counter-calibration runs instead of the benchmark: 'flops' integrates "
                         "every lane of full waves for a fixed number of fixed steps (FP64 "
                         "instruction counters per lane-step); 'copy' streams a buffer of "
                         "known size (HBM byte counters); 'mlp' times the proposal network's "
                         "forward and gradient kernels at a large batch")
    ap.add_argument("--probe-lanes", type=int, default=256 * 1024)
    ap.add_argument("--probe-steps", type=int, default=300)
    ap.add_argument("--probe-h", type=float, default=0.5)
    ap.add_argument("--probe-mib", type=int, default=1024)
    ap.add_argument("--probe-mlp-rows", type=int, default=1 << 20)
    return ap.parse_args()


def _oracle_sample(wl, stride):
    """Every stride-th trajectory of the workload, counted over all its
    trajectories in instance order (a systematic sample spread over every
    instance), as global ids per instance."""
    import numpy as np
    out, pos = [], 0
    for i in wl.instances:
        first = (-pos) % stride                  # first local index on the global stride
        out.append(np.arange(i.first_id + first, i.first_id + i.n_traj, stride, dtype=np.int64))
        pos += i.n_traj
    return out


def cpu_baseline(wl, stride_pool, stride_one, procs):
    """The oracle as it stands on the host cores, on stratified samples of
    the same workload (every k-th trajectory id of every instance): a process
    pool of `procs` copies, and one core alone (time per trajectory and trial
    steps per second)."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    per = _oracle_sample(wl, stride_pool)
    n = int(sum(len(p) for p in per))
    t0 = time.perf_counter()
    recs, _ = oracle.run_workload(wl, per, processes=procs)
    dt = time.perf_counter() - t0
    per1 = _oracle_sample(wl, stride_one)
    n1 = int(sum(len(p) for p in per1))
    t1 = time.perf_counter()
    recs1, _ = oracle.run_workload(wl, per1, processes=1)
    dt1 = time.perf_counter() - t1
    steps1 = int(recs1["nstep"].sum() + recs1["nrej"].sum())
    cpu = host_cpu()
    return {"value": n / dt, "unit": "trajectories/s", "cores": procs, "kind": "oracle",
            "sample": "every %dth trajectory over all %d instances (%d trajectories), serial C "
                      "oracle in a %d-process pool, %.1f s, on %s"
                      % (stride_pool, len(wl.instances), n, procs, dt, cpu),
            "one_core": {"trajectories_per_s": n1 / dt1, "ms_per_trajectory": 1e3 * dt1 / n1,
                         "trial_steps_per_s": steps1 / dt1,
                         "sample": "every %dth trajectory over all %d instances (%d "
                                   "trajectories, %d trial steps), one process, %.1f s"
                                   % (stride_one, len(wl.instances), n1, steps1, dt1)}}


def host_cpu() -> str:
    """Model and logical CPU count of the host."""
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return "%s (%d logical CPUs)" % (model, os.cpu_count() or 0)


def probe_flops(args, W, Q, torch):
    """Every lane of full waves integrates exactly probe_steps fixed steps of
    the one-lane propagation kernel (no lane finishes early, no rejections),
    so the FP64 instruction counters divided by the lane-steps give the FP64
    work of one trial step."""
    import numpy as np
    wl = W.CONFIGS[args.workload]()
    prm = dataclasses.replace(wl.params, fixed_step=1, h_fixed=args.probe_h, rk=RK_NAMES[args.rk])
    ctx = Q.Context(wl.system, prm, device=0)
    ctx.set_instances(wl.instances)
    n = args.probe_lanes
    ids = (torch.arange(n, dtype=torch.int64, device="cuda:0") % wl.n_traj).contiguous()
    st = ctx.new_state(n)
    ctx.init_conditions(ids, st)
    # every lane: exactly probe_steps + 1 steps of size h (the last one
    # reaches t_max), no distance stop
    st.d[Q.F_TMAX].fill_(args.probe_steps * args.probe_h * (1 + 1e-12))
    st.d[Q.F_RSTOP].fill_(1e9)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.propagate(st)
    e1.record()
    torch.cuda.synchronize()
    ns = st.nstep.cpu().numpy()
    return {"probe": "flops", "workload": wl.name, "rk": args.rk, "lanes": n,
            "steps_min": int(ns.min()), "steps_max": int(ns.max()),
            "lane_steps": int(ns.astype(np.int64).sum()), "kernel_ms": e0.elapsed_time(e1)}


def probe_copy(args, torch):
    """y = -x over probe_mib MiB of FP64, three launches: each reads and
    writes exactly that many bytes, for scaling FETCH_SIZE and WRITE_SIZE."""
    n = args.probe_mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    return {"probe": "copy", "bytes_read_per_launch": n * 8, "bytes_written_per_launch": n * 8,
            "launches": 3}


def probe_mlp(args, Q, torch):
    """The proposal network's kernels at large batches: the forward pass on
    probe_mlp_rows rows of synthetic features, and the gradient (forward,
    backward, one weight-gradient partial per 64-row workgroup and their
    fixed-order reduction) on the training batch (4096 rows) and on 65,536
    rows; three timed calls each after one untimed, HIP events on the
    current stream.  Algorithmic work per row: 68,096 FLOP forward
    (6-128-128-128-4 matrix products), three times that for the gradient."""
    g = torch.Generator(device="cuda:0")
    g.manual_seed(5)
    net = Q.MLP(seed=11, device=0)
    flop_fwd = 2 * (6 * 128 + 128 * 128 + 128 * 128 + 128 * 4)
    out = {"probe": "mlp", "flop_per_row_forward": flop_fwd}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 3

    for name, n, mult in (("forward", args.probe_mlp_rows, 1), ("gradient_4096", 4096, 3),
                          ("gradient_65536", 65536, 3)):
        x = torch.rand((n, Q.MLP_NIN), dtype=torch.float32, device="cuda:0", generator=g)
        y = torch.randint(0, Q.MLP_NOUT, (n,), dtype=torch.int32, device="cuda:0", generator=g)
        fn = (lambda: net.forward(x)) if mult == 1 else (lambda: net.gradient(x, y))
        ms = timed(fn)
        tf = mult * flop_fwd * n / (ms * 1e-3) / 1e12
        out[name] = {"rows": n, "ms": ms, "tflops": tf, "frac_bf16_dense_peak": tf / 2500.0}
    return out


def outcomes_by_status(np, lab, status):
    """Counts of each outcome label by the stop status that ended the
    trajectory (nonzero entries only)."""
    out = {}
    for l, ln in enumerate(LABEL_NAMES):
        m = lab == l
        if not m.any():
            continue
        c = np.bincount(status[m], minlength=len(STATUS_NAMES))
        out[ln] = {STATUS_NAMES[k]: int(c[k]) for k in range(len(STATUS_NAMES)) if c[k]}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(trajectories shard by id range; see the design notes)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import qcams_workloads as W
    import paper_2304_02731_amd as Q

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.probe != "none":
        res = (probe_flops(args, W, Q, torch) if args.probe == "flops" else
               probe_mlp(args, Q, torch) if args.probe == "mlp" else probe_copy(args, torch))
        print(json.dumps(res), flush=True)
        return
    wl = W.CONFIGS[args.workload]()
    surface, stride_pool, stride_one = WORKLOADS[args.workload]
    rk = RK_NAMES[args.rk]
    # the Sec. 3.1 example tolerances where this integrator keeps the energy
    # gate on this workload, else the Sec. 3.4 timing-study tolerances
    wl.params = W.gated_params(wl, rk)
    if args.atol is not None:
        wl.params = dataclasses.replace(wl.params, atol=args.atol)
    if args.rtol is not None:
        wl.params = dataclasses.replace(wl.params, rtol=args.rtol)
    ctx = Q.Context(wl.system, wl.params, device=0)
    ctx.set_instances(wl.instances)
    stream = torch.cuda.Stream()
    opts = Q.RunOpts(blocks=args.blocks, refill_min=args.refill_min,
                     check_every=args.check_every, lpt=0 if args.no_lpt else 1,
                     graph=0 if args.no_graph else 1, lanes=args.lanes)
    tuned = None
    with torch.cuda.stream(stream):
        buf = ctx.new_run_buffers()
        if args.autotune:
            best, best_ms = ctx.autotune(buf, reps=1)
            best.graph = opts.graph
            opts = best
            tuned = {"opts": best.as_dict(), "ms": best_ms}
        ids = ctx.all_ids()
    n = ids.numel()
    st, out = buf["state"], buf["outcome"]
    prop_times = []
    grid_groups = ctx.grid_groups()[0]
    grid_out = []

    def step(timed):
        # units and levels of every instance (a1, a2), then the path (a3-a9)
        ctx.set_instances(wl.instances)
        if args.path == "run":
            ctx.run(buf, opts, stream=stream)
            if grid_groups:
                grid_out.append(ctx.grid_cross_sections(buf["xs"], stream=stream))
        else:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            ctx.init_conditions(ids, st, buf["sample"], stream=stream)
            e0.record(stream)
            ctx.propagate(st, stream=stream)
            e1.record(stream)
            ctx.classify(st, out, stream=stream)
            ctx.cross_sections(out, ids, stream=stream)
        if timed:
            # duration of the propagation kernel: HIP events on its stream
            prop_times.append(ctx.last_run_kernel_ms() if args.path == "run"
                              else (e0, e1))

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            step(False)
            print("warm-up step done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(args.steps):
            step(True)
            print("step done", file=sys.stderr, flush=True)
        ev1.record(stream)
        torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    prop_ms = float(np.mean([t if isinstance(t, float) else t[0].elapsed_time(t[1])
                             for t in prop_times]))

    used = ctx.last_run_options() if args.path == "run" else None
    # work of the last step
    nstep = st.nstep.cpu().numpy().astype(np.int64)
    nrej = st.nrej.cpu().numpy().astype(np.int64)
    per_traj = nstep + nrej
    trial_steps = int(per_traj.sum())
    fs = F_STEP[(surface, rk)]
    rate = trial_steps / (prop_ms * 1e-3)            # trial steps per second
    achieved = rate * fs["hand"] / 1e12
    slots = None
    if args.path == "run":
        # how full the persistent waves' slots were over their trial-step loop
        wave_steps = ctx.last_run_wave_steps()
        spw = 64 // used.lanes
        slots = {"wave_steps": wave_steps, "slots_per_wave": spw,
                 "slot_utilization": trial_steps / (wave_steps * spw) if wave_steps else None}
    lab = out.label.cpu().numpy()
    status = st.status.cpu().numpy()
    dE = out.d[3].cpu().numpy()
    fin = lab != Q.FAILED
    kernel = ("k_persistent<%d,%s,%d>" % (used.lanes, KINDS[surface], rk) if args.path == "run"
              else "k_propagate<%s,%d>" % (KINDS[surface], rk))
    peak = PEAK_FP64_VECTOR / 1e12
    res = {
        "metric": "QCT trajectories/s (FP64, H2+Ca)",
        "value": n / (ms_step * 1e-3),
        "unit": "trajectories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_traj": n, "instances": len(wl.instances),
                   "surface": wl.system.name, "integrator": args.rk, "atol": wl.params.atol,
                   "rtol": wl.params.rtol, "R0": wl.params.R0, "t_stop": wl.params.t_stop,
                   "r_stop": wl.params.r_stop},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": TRAFFIC.get((wl.name, kernel)),
                     "kernel": kernel, "timed_ms": prop_ms, "trial_steps": trial_steps,
                     "flop_per_trial_step": fs["hand"],
                     "flop_per_trial_step_hand": fs["hand"], "frac_hand": achieved / peak,
                     "flop_per_trial_step_method": fs["method"],
                     "frac_method": rate * fs["method"] / PEAK_FP64_VECTOR,
                     "flop_per_trial_step_counter": fs["counter"],
                     "frac_counter": (rate * fs["counter"] / PEAK_FP64_VECTOR
                                      if fs["counter"] is not None else None)},
        "path": args.path, "run_opts": used.as_dict() if used else opts.as_dict(),
        "slots": slots,
        "autotune": tuned,
        "trial_steps_per_s": trial_steps / (ms_step * 1e-3),
        "trial_steps_per_traj": {q: int(np.percentile(per_traj, p)) for q, p in
                                 (("p50", 50), ("p90", 90), ("p99", 99), ("p999", 99.9),
                                  ("max", 100))},
        "max_abs_dE_rel": float(np.abs(dE[fin]).max()) if fin.any() else None,
        "energy_gate": {"limit": 1e-8,
                        "passed": bool(fin.any() and np.abs(dE[fin]).max() < 1e-8)},
        "labels": np.bincount(lab, minlength=6).tolist(),
        "outcomes_by_status": outcomes_by_status(np, lab, status),
        "wall_s": wall,
    }
    if res["roofline"]["traffic"]:
        # HBM bandwidth the propagation kernel draws, beside its FP64 rate
        res["roofline"]["hbm_GB_per_s"] = res["roofline"]["traffic"] / (prop_ms * 1e-3) / 1e9
    if grid_out:
        g = grid_out[-1].cpu().numpy()
        res["grid"] = {"E_c_K": g[:, Q.G_EC].tolist(),
                       "sigma_a0^2 [q, r1, r2, d]": g[:, Q.G_SIGMA:Q.G_SIGMA + 4].tolist(),
                       "sigma_err": g[:, Q.G_DSIGMA:Q.G_DSIGMA + 4].tolist(),
                       "rate_au [q, r1, r2, d]": g[:, Q.G_RATE:Q.G_RATE + 4].tolist()}
    if not args.no_learned:
        res["learned"] = learned_metric(args)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(wl, args.cpu_stride or stride_pool, stride_one,
                                           args.cpu_procs)
    print(json.dumps(res), flush=True)


def learned_metric(args):
    """Train on 2e5 trajectories of the batched workload (GPU), then compare
    the dissociation cross section's variance x GPU-seconds, plain against
    importance-sampled, over seeded replicates."""
    import qcams_workloads as W
    import paper_2304_02731_amd as Q
    from paper_2304_02731_amd import learned as L
    tw = W.config_learned_train()
    tr = L.train_network(tw.system, tw.params, tw.instances, epochs=args.learned_epochs)
    print("learned: trained (%d rows, %.2f s data, %.2f s training, val CE %.4f, prior CE %.4f)"
          % (tr.n_train, tr.data_s, tr.train_s, tr.val_loss, tr.prior_loss), file=sys.stderr,
          flush=True)
    tgt = W.config_learned_target(n_traj=args.learned_n).instances[0]
    c = L.compare(tw.system, tw.params, tgt, None if tr.fallback else tr.net, channel=Q.DISS,
                  n=args.learned_n, replicates=args.learned_replicates)
    print("learned: compared (%d replicates)" % args.learned_replicates, file=sys.stderr,
          flush=True)
    return {"metric": "var(sigma_diss) x GPU-s, plain / learned", "value": c.efficiency,
            "ci95": list(c.efficiency_ci95), "target_min": 5.0,
            "target": "H2(v=4,j=0)+Ca, 5e4 K, b by area to 10 a0, dissociation",
            "n_per_replicate": args.learned_n, "replicates": args.learned_replicates,
            "sigma_plain": float(c.sigma_plain[Q.DISS]), "sigma_learned": float(c.sigma_is[Q.DISS]),
            "var_plain": c.var_plain, "var_learned": c.var_is, "gpu_s_plain": c.gpu_s_plain,
            "gpu_s_learned": c.gpu_s_is, "proposal_build_s": c.proposal_s, "ess_per_draw": c.ess,
            "fallback_to_plain": c.fallback, "train_rows": tr.n_train,
            "train_loss_first_last": [tr.train_loss[0], tr.train_loss[-1]],
            "val_ce": tr.val_loss, "prior_ce": tr.prior_loss, "train_s": tr.train_s,
            "data_s": tr.data_s}


if __name__ == "__main__":
    main()
