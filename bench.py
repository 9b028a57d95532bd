#!/usr/bin/env python3
"""Benchmark of the QCT hot path on one MI355X.

One step = one pass of the whole path over the batched H2 + Ca workload
(96 instances: 16 collision energies 1e3..1e5 K x v in {0,2,4} x j in {0,5},
1042 trajectories each, b uniform in area to 10 a0; 100,032 trajectories):
instance set-up with Bohr-Sommerfeld levels, initial conditions, adaptive
Runge-Kutta propagation (Dormand-Prince 5(4), the paper's integrator, or the
8(5,3) variant) of every trajectory to its stop rule, classification and
Gaussian binning, per-instance cross sections and rates.  All inputs are
synthetic and seeded; nothing is cached between steps.

Prints one JSON line (metric, value, roofline of the propagation kernel,
CPU-oracle baseline on a bounded sample).
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

# FP64 operations per trial step of one trajectory (FMA = 2), counted with
# hardware FP64 instruction counters on a full-wave fixed-step run of the
# one-lane propagation kernel, per surface and RK variant.
F_STEP = {("morse", 0): 1833.7, ("morse", 1): 3996.7,
          ("mixed", 0): 1719.6, ("mixed", 1): 3768.6}
# HBM bytes per launch of the persistent kernel from FETCH_SIZE and WRITE_SIZE
# passes scaled by a streaming kernel of known size, for the kernel as it was
# when the counters were taken (workload, kernel) -> bytes; null otherwise.
TRAFFIC = {("batched", "k_persistent<4,0,0,0,1>"): 32.70e6}
RK_NAMES = {"dopri5": 0, "dop853": 1}
KINDS = {"morse": "0,0,0", "mixed": "3,0,2"}   # 3: LJ 12-6 specialisation
# workload -> (surface, default CPU-baseline stride)
WORKLOADS = {"batched": ("morse", 2), "small": ("morse", 1), "mixed": ("mixed", 500),
             "sweep": ("morse", 5000), "paper_grid": ("morse", 1000)}
PEAK_FP64_VECTOR = 78.6e12   # MI355X, FLOP/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batched", choices=list(WORKLOADS))
    ap.add_argument("--cpu-stride", type=int, default=0,
                    help="CPU baseline runs every k-th trajectory id through the oracle "
                         "(0: the workload's default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-procs", type=int, default=16)
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
    ap.add_argument("--learned", action="store_true",
                    help="also train the proposal network and report variance x GPU-seconds, "
                         "learned vs plain, for dissociation of H2(v=4,j=0)+Ca at 5e4 K")
    ap.add_argument("--learned-replicates", type=int, default=96)
    ap.add_argument("--learned-n", type=int, default=200_000)
    ap.add_argument("--learned-epochs", type=int, default=20)
    return ap.parse_args()


def cpu_baseline(wl, stride, procs):
    """The oracle as it stands on the host cores, on a stratified sample of
    the same workload (every stride-th trajectory id of every instance)."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    per = [np.arange(i.first_id, i.first_id + i.n_traj, stride, dtype=np.int64)
           for i in wl.instances]
    n = int(sum(len(p) for p in per))
    t0 = time.perf_counter()
    recs, _ = oracle.run_workload(wl, per, processes=procs)
    dt = time.perf_counter() - t0
    nth = {1: "", 2: "2nd ", 3: "3rd "}.get(stride, "%dth " % stride)
    return {"value": n / dt, "unit": "trajectories/s", "cores": procs, "kind": "oracle",
            "sample": "every %strajectory id of all %d instances (%d trajectories), "
                      "serial C oracle in a %d-process pool, %.1f s, on %s"
                      % (nth, len(wl.instances), n, procs, dt, host_cpu())}


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
    wl = W.CONFIGS[args.workload]()
    surface, stride = WORKLOADS[args.workload]
    rk = RK_NAMES[args.rk]
    # the Sec. 3.1 example tolerances where this integrator keeps the energy
    # gate on this workload, else the Sec. 3.4 timing-study tolerances
    wl.params = W.gated_params(wl, rk)
    if args.atol is not None:
        wl.params = dataclasses.replace(wl.params, atol=args.atol)
    if args.rtol is not None:
        wl.params = dataclasses.replace(wl.params, rtol=args.rtol)
    dev = torch.device("cuda", 0)
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
    f_step = F_STEP[(surface, rk)]
    achieved = trial_steps * f_step / (prop_ms * 1e-3) / 1e12 if f_step else None
    slots = None
    if args.path == "run":
        # how full the persistent waves' slots were over their trial-step loop
        wave_steps = ctx.last_run_wave_steps()
        spw = 64 // used.lanes
        slots = {"wave_steps": wave_steps, "slots_per_wave": spw,
                 "slot_utilization": trial_steps / (wave_steps * spw) if wave_steps else None}
    lab = out.label.cpu().numpy()
    dE = out.d[3].cpu().numpy()
    fin = lab != Q.FAILED
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
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_VECTOR / 1e12,
                     "unit": "TFLOP/s",
                     "frac": achieved * 1e12 / PEAK_FP64_VECTOR if achieved else None,
                     "traffic": None,   # filled below
                     "kernel": ("k_persistent<%d,%s,%d>" % (used.lanes, KINDS[surface], rk)
                                if args.path == "run"
                                else "k_propagate<%s,%d>" % (KINDS[surface], rk)),
                     "timed_ms": prop_ms, "trial_steps": trial_steps,
                     "flop_per_trial_step": f_step},
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
        "wall_s": wall,
    }
    res["roofline"]["traffic"] = TRAFFIC.get((args.workload, res["roofline"]["kernel"]))
    if res["roofline"]["traffic"]:
        # HBM bandwidth the propagation kernel draws, beside its FP64 rate
        res["roofline"]["hbm_GB_per_s"] = res["roofline"]["traffic"] / (prop_ms * 1e-3) / 1e9
    if grid_out:
        g = grid_out[-1].cpu().numpy()
        res["grid"] = {"E_c_K": g[:, Q.G_EC].tolist(),
                       "sigma_a0^2 [q, r1, r2, d]": g[:, Q.G_SIGMA:Q.G_SIGMA + 4].tolist(),
                       "sigma_err": g[:, Q.G_DSIGMA:Q.G_DSIGMA + 4].tolist(),
                       "rate_au [q, r1, r2, d]": g[:, Q.G_RATE:Q.G_RATE + 4].tolist()}
    if args.learned:
        res["learned"] = learned_metric(args)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(wl, args.cpu_stride or stride, args.cpu_procs)
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
    return {"metric": "var(sigma_diss) x GPU-s, plain / learned", "value": c.efficiency,
            "ci95": list(c.efficiency_ci95),
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
