"""Full-wave run of the propagation kernel for counting FP64 work per step.

Every lane integrates the same number of fixed-size steps of the chosen RK
variant (no lane finishes early, no rejections), so hardware FP64
instruction counters divided by (lanes x steps) give the FP64 operations of
one trial step.  Run under
``rocprofv3 --pmc SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64
SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_TRANS_F64``.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--lanes", type=int, default=256 * 1024)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--h", type=float, default=0.25)
    ap.add_argument("--rk", type=int, default=0, help="0: DOPRI5, 1: DOP853")
    ap.add_argument("--workload", default="batched", choices=["batched", "mixed"])
    args = ap.parse_args()
    import torch

    import qcams_workloads as W
    import paper_2304_02731_amd as Q

    wl = W.CONFIGS[args.workload]()
    prm = dataclasses.replace(wl.params, fixed_step=1, h_fixed=args.h, rk=args.rk)
    ctx = Q.Context(wl.system, prm, device=0)
    ctx.set_instances(wl.instances)
    n = args.lanes
    ids = (torch.arange(n, dtype=torch.int64, device="cuda:0") % wl.n_traj).contiguous()
    st = ctx.new_state(n)
    ctx.init_conditions(ids, st)
    # every lane: exactly `steps` steps of size h, no distance stop
    st.d[Q.F_TMAX].fill_(args.steps * args.h * (1 + 1e-12))
    st.d[Q.F_RSTOP].fill_(1e9)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.propagate(st)
    e1.record()
    torch.cuda.synchronize()
    ns = st.nstep.cpu()
    print(json.dumps({"workload": wl.name, "rk": args.rk, "lanes": n, "steps_min": int(ns.min()), "steps_max": int(ns.max()),
                      "lane_steps": int(ns.sum()), "kernel_ms": e0.elapsed_time(e1)}), flush=True)


if __name__ == "__main__":
    main()
