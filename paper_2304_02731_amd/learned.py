"""Learned importance-sampling proposal: training data from the method
itself, GPU training of the network, the proposal for a target instance and
channel, and the variance-per-GPU-second comparison with plain sampling.

Every step runs in the library's kernels (trajectory runs, features, BF16
forward/backward, Adam, proposal tables, weighted reductions); this module
only orders the calls, draws the minibatch permutations (seeded numpy) and
does the scalar bookkeeping of the comparison.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Optional

import numpy as np

from . import qcams as Q


@dataclasses.dataclass
class TrainResult:
    net: "Q.MLP"
    train_loss: list
    val_loss: float
    prior_loss: float
    n_train: int
    n_val: int
    data_s: float
    train_s: float
    fallback: bool


def _prior_ce(y: np.ndarray) -> float:
    """Cross-entropy of the class frequencies (the network must beat it)."""
    f = np.bincount(y, minlength=4) / len(y)
    f = f[f > 0]
    return float(-(f * np.log(f)).sum())


def train_network(system, params, instances, epochs: int = 20, batch: int = 4096,
                  lr: float = 1e-3, seed: int = 7, val_frac: float = 0.1,
                  stream=None) -> TrainResult:
    """Run the training workload, build (x, y) on the GPU and train."""
    import torch
    ctx = Q.Context(system, params)
    ctx.set_instances(instances)
    buf = ctx.new_run_buffers()
    t0 = time.perf_counter()
    ctx.run(buf, Q.RunOpts(blocks=0, refill_min=1, check_every=8, lpt=1, graph=0), stream=stream)
    x, y = ctx.mlp_features(buf["ids"], buf["sample"], buf["outcome"], stream=stream)
    torch.cuda.synchronize()
    data_s = time.perf_counter() - t0
    yh = y.cpu().numpy()
    rows = np.nonzero(yh >= 0)[0]
    rng = np.random.default_rng(seed)
    rng.shuffle(rows)
    nval = max(1, int(val_frac * len(rows)))
    val, tr = rows[:nval], rows[nval:]
    ntr = (len(tr) // batch) * batch
    tr = tr[:ntr]
    net = Q.MLP(seed=seed)
    dev = ctx.torch_device
    perm_d = torch.zeros(ntr, dtype=torch.int32, device=dev)
    loss_d = torch.zeros(1, dtype=torch.float32, device=dev)
    losses = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm_d.copy_(torch.as_tensor(rng.permutation(tr).astype(np.int32)))
        net.train_epoch(x, y, perm_d, batch, lr, loss_d, stream=stream)
        losses.append(loss_d.item() / (ntr // batch))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    vidx = torch.as_tensor(val.astype(np.int32), device=dev)
    _, vloss = net.gradient(x, y, idx=vidx)
    vl = vloss.item()
    prior = _prior_ce(yh[val])
    return TrainResult(net, losses, vl, prior, ntr, nval, data_s, train_s, fallback=vl >= prior)


def ess_fraction(q: np.ndarray) -> float:
    """Effective sample size per sample of the cell proposal, (E_q w)^2/E_q w^2
    with w_k = (1/K)/q_k."""
    K = len(q)
    Ew2 = float(np.sum(1.0 / (K * K * q)))
    return 1.0 / Ew2


@dataclasses.dataclass
class Comparison:
    sigma_plain: np.ndarray
    sigma_is: np.ndarray
    var_plain: float
    var_is: float
    gpu_s_plain: float
    gpu_s_is: float
    proposal_s: float
    efficiency: float
    efficiency_ci95: tuple    # from the F distribution of the variance ratio
    ess: float
    fallback: bool
    channel: int


def _replicates(system, params, inst_template, n, seeds, mode, stream, proposal=None):
    import torch
    sig, se, ms = [], [], []
    for s in seeds:
        inst = dataclasses.replace(inst_template, n_traj=n, first_id=0, seed=int(s), b_mode=mode)
        ctx = Q.Context(system, params)
        ctx.set_instances([inst])
        if proposal is not None:
            ctx.proposal_set(proposal)
        buf = ctx.new_run_buffers()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.run(buf, Q.RunOpts(blocks=0, refill_min=1, check_every=8, lpt=1, graph=0))
        e1.record()
        torch.cuda.synchronize()
        xs = buf["xs"].cpu().numpy()[0]
        sig.append(xs[Q.XS_SIGMA:Q.XS_SIGMA + 4].copy())
        se.append(xs[Q.XS_DSIGMA:Q.XS_DSIGMA + 4].copy())
        ms.append(e0.elapsed_time(e1))
        ctx.close()
    return np.array(sig), np.array(se), np.array(ms) / 1e3


def compare(system, params, target, net: Optional["Q.MLP"], channel: int = Q.DISS,
            n: int = 200_000, replicates: int = 16, alpha: float = 0.1,
            seed0: int = 1000) -> Comparison:
    """Variance x GPU-seconds of the channel's cross section, plain sampling
    against the learned proposal, over seeded replicates (Var = replicate
    variance of sigma).  The proposal falls back to plain sampling when its
    effective sample size per draw is below 0.1."""
    import torch
    t0 = time.perf_counter()
    ctx = Q.Context(system, params)
    ctx.set_instances([dataclasses.replace(target, b_mode=Q.B_PROPOSAL)])
    q = ctx.proposal_build(net, 0, channel, alpha if net is not None else 1.0)
    torch.cuda.synchronize()
    prop_s = time.perf_counter() - t0
    qh = q.cpu().numpy()
    ctx.close()
    ess = ess_fraction(qh)
    fallback = net is None or ess < 0.1
    seeds_p = seed0 + np.arange(replicates)
    seeds_i = seed0 + 10_000 + np.arange(replicates)
    sp, _, tp = _replicates(system, params, target, n, seeds_p, Q.B_AREA, None)
    if fallback:
        si, ti = sp, tp
    else:
        si, _, ti = _replicates(system, params, target, n, seeds_i, Q.B_PROPOSAL, None, proposal=qh)
    vp = float(np.var(sp[:, channel], ddof=1))
    vi = float(np.var(si[:, channel], ddof=1))
    Tp, Ti = float(tp.mean()), float(ti.mean()) + (0.0 if fallback else prop_s / replicates)
    eff = (vp * Tp) / (vi * Ti) if vi > 0 else float("inf")
    # the ratio of two sample variances of normal replicates, each with
    # replicates - 1 degrees of freedom, scaled by the true ratio is F-distributed
    from scipy import stats
    dof = replicates - 1
    lo, hi = stats.f.ppf([0.025, 0.975], dof, dof)
    ci = (eff / hi, eff / lo) if vi > 0 else (float("inf"), float("inf"))
    return Comparison(sp.mean(axis=0), si.mean(axis=0), vp, vi, Tp, Ti, prop_s, eff, ci, ess,
                      fallback, channel)
