"""Input files in the paper's JSON layout and its two CSV outputs.

Input (Sec. 3.1, Listing 1): keys ``vi``, ``ji``, ``Ec (K)``, ``b``, ``r0``,
``seed``, ``potential_AB`` / ``_BC`` / ``_CA`` (``morse`` | ``lj`` |
``buck``), ``masses`` {``ma``, ``mb``, ``mc``} in electron masses,
``int_params`` {``t_stop``, ``r_stop``, ``a_tol``, ``r_tol``} and
``potential_params`` {``AB``, ``BC``, ``CA``}, each with the parameters of
the three families (Sec. 3.2): Morse {``de``, ``re``, ``we``}, generalized
LJ {``m``, ``n``, ``cm``, ``cn``, ``re``}, Buckingham {``a``, ``b``, ``c6``,
``re``, ``max``}, and the DVR grid {``npts``, ``xmin``, ``xmax``}.  All in
atomic units except the collision energy (kelvin).  The Morse pairs are
handed to the library by their harmonic frequency (the library takes the
range parameter alpha = w_e sqrt(mu / (2 D_e)) with mu the pair's reduced
mass, qcams_system_resolve).  The ``re`` and ``max`` guesses are kept
but not needed: the library finds the pair shapes itself.  The DVR grid of
pair AB serves when a run asks for DVR levels (``levels="dvr"``).  A null
seed is replaced by one drawn from the operating system and reported.

Outputs (Sec. 3.3): the short form has one row per (E_c, b) with the summed
product counts; the long form one row per trajectory with its product
count vector n_f, final state s_f = (v_t, w, j_t) ((0, 0, 0) unless exactly
one pair is bound), final rho_1, rho_2, P_1, P_2, final time, and the random
draws that recreate it.

This module only reads and writes; every trajectory runs in the library's
kernels (``Context.run``).
"""
from __future__ import annotations

import argparse
import csv
import dataclasses
import json
import os
from typing import Optional, Sequence

import numpy as np

from . import qcams as Q

KINDS = ("morse", "lj", "buck")


@dataclasses.dataclass(frozen=True)
class Pair:
    kind: str
    params: dict


@dataclasses.dataclass(frozen=True)
class System:
    """A system in electron masses (what the input file holds)."""
    masses_me: tuple
    pairs: tuple
    name: str = "input file"


@dataclasses.dataclass
class Calc:
    system: System
    params: object            # qcams_workloads.Params-like
    v: int
    j: int
    Ec_K: float
    b: float
    seed: int
    seed_from_file: bool
    dvr: dict                 # per pair: npts, xmin, xmax (AB's used for DVR levels)
    guesses: dict             # per pair: re / max guesses (kept, unused)


def _pair(kind: str, p: dict) -> Pair:
    if kind == "morse":
        return Pair("morse", {"De": float(p["de"]), "re": float(p["re"]), "we": float(p["we"])})
    if kind == "lj":
        return Pair("lj", {"n": int(p["n"]), "m": int(p["m"]), "Cn": float(p["cn"]),
                           "Cm": float(p["cm"])})
    if kind == "buck":
        return Pair("buck", {"A": float(p["a"]), "b": float(p["b"]), "C6": float(p["c6"])})
    raise ValueError("unknown potential %r (expected one of %s)" % (kind, ", ".join(KINDS)))


def load_input(src) -> Calc:
    """Read an input file (path, JSON text or dict) in the paper's layout."""
    import qcams_workloads as W
    if isinstance(src, dict):
        d = src
    elif isinstance(src, str) and src.lstrip().startswith("{"):
        d = json.loads(src)
    else:
        with open(src) as f:
            d = json.load(f)
    m = d["masses"]
    ma, mb, mc = float(m["ma"]), float(m["mb"]), float(m["mc"])
    pairs, dvr, guesses = [], {}, {}
    for name in ("AB", "BC", "CA"):
        kind = d["potential_" + name]
        pp = d["potential_params"][name]
        pairs.append(_pair(kind, pp[kind]))
        dvr[name] = {k: pp[k] for k in ("npts", "xmin", "xmax") if k in pp}
        guesses[name] = {k: pp[kind][k] for k in ("re", "max") if k in pp[kind]}
    ip = d.get("int_params", {})
    base = W.Params()
    params = dataclasses.replace(
        base, R0=float(d.get("r0", base.R0)), t_stop=float(ip.get("t_stop", base.t_stop)),
        r_stop=float(ip.get("r_stop", base.r_stop)), atol=float(ip.get("a_tol", base.atol)),
        rtol=float(ip.get("r_tol", base.rtol)))
    seed = d.get("seed")
    from_file = seed is not None
    if seed is None:
        seed = int.from_bytes(os.urandom(8), "little") >> 1
    return Calc(System((ma, mb, mc), tuple(pairs)), params, int(d["vi"]), int(d["ji"]),
                float(d["Ec (K)"]), float(d.get("b", 0.0)), int(seed), from_file, dvr, guesses)


def run(calc: Calc, n_traj: int, b_values: Optional[Sequence[float]] = None,
        device: int = 0, rk: Optional[int] = None, opts: Optional["Q.RunOpts"] = None,
        levels: str = "bs"):
    """Run n_traj trajectories at each impact parameter (default: the file's
    b) in one fused launch.  levels: "bs" (Bohr-Sommerfeld) or "dvr" (the
    file's DVR grid of pair AB).  Returns a dict of host arrays: the
    instance rows (E_c, b), per-instance result rows, and per-trajectory
    outputs."""
    import qcams_workloads as W
    bs = [calc.b] if b_values is None else [float(b) for b in b_values]
    params = calc.params if rk is None else dataclasses.replace(calc.params, rk=rk)
    inst = [W.Instance(calc.Ec_K, calc.v, calc.j, n_traj, k * n_traj, calc.seed, W.B_FIXED, b, 0.0)
            for k, b in enumerate(bs)]
    ctx = Q.Context(calc.system, params, device=device, masses_me=calc.system.masses_me)
    if levels == "dvr":
        g = calc.dvr["AB"]
        ctx.set_level_method(Q.LEVELS_DVR, int(g["npts"]), float(g["xmin"]), float(g["xmax"]))
    elif levels != "bs":
        raise ValueError("levels must be 'bs' or 'dvr'")
    ctx.set_instances(inst)
    buf = ctx.new_run_buffers()
    ctx.run(buf, opts)
    import torch
    torch.cuda.synchronize()
    res = {
        "instances": inst,
        "xs": buf["xs"].cpu().numpy(),
        "ids": buf["ids"].cpu().numpy(),
        "state": buf["state"].d.cpu().numpy(),
        "status": buf["state"].status.cpu().numpy(),
        "label": buf["outcome"].label.cpu().numpy(),
        "vt": buf["outcome"].vt.cpu().numpy(),
        "jt": buf["outcome"].jt.cpu().numpy(),
        "out": buf["outcome"].d.cpu().numpy(),
        "sample": buf["sample"].cpu().numpy(),
    }
    ctx.close()
    return res


SHORT_COLUMNS = ["Ec (K)", "b", "N", "N_q", "N_r1", "N_r2", "N_d", "N_unresolved", "N_failed"]
LONG_COLUMNS = (["Ec (K)", "b", "v", "j", "id", "n_q", "n_r1", "n_r2", "n_d", "v_t", "w", "j_t"]
                + ["rho1_x", "rho1_y", "rho1_z", "rho2_x", "rho2_y", "rho2_z",
                   "P1_x", "P1_y", "P1_z", "P2_x", "P2_y", "P2_z", "t_f"]
                + ["cos_theta", "phi", "eta", "chi", "seed", "dE_rel", "status"])


def _open(path: str, header: Sequence[str], append: bool):
    exists = append and os.path.exists(path) and os.path.getsize(path) > 0
    f = open(path, "a" if append else "w", newline="")
    w = csv.writer(f)
    if not exists:
        w.writerow(header)
    return f, w


def write_short(path: str, res: dict, append: bool = True) -> int:
    """One row per (E_c, b): the summed product counts.  Returns rows written."""
    f, w = _open(path, SHORT_COLUMNS, append)
    with f:
        for k, I in enumerate(res["instances"]):
            row = res["xs"][k]
            c = [int(round(x)) for x in row[Q.XS_COUNTS:Q.XS_COUNTS + 6]]
            w.writerow([repr(I.Ec_K), repr(I.b), int(round(row[Q.XS_N]))] + c)
    return len(res["instances"])


def write_long(path: str, res: dict, append: bool = True) -> int:
    """One row per trajectory (natural order: instances, then ids)."""
    f, w = _open(path, LONG_COLUMNS, append)
    inst = res["instances"]
    firsts = np.array([I.first_id for I in inst])
    with f:
        for p in range(len(res["ids"])):
            tid = int(res["ids"][p])
            I = inst[int(np.searchsorted(firsts, tid, side="right") - 1)]
            lab = int(res["label"][p])
            nf = [1 if lab == c else 0 for c in range(4)]
            single = lab < 3
            sf = ([int(res["vt"][p]), float(res["out"][2, p]), int(res["jt"][p])] if single
                  else [0, 0.0, 0])
            y = res["state"][:13, p].tolist()
            smp = res["sample"][1:5, p].tolist()
            w.writerow([repr(I.Ec_K), repr(I.b), I.v, I.j, tid] + nf + sf + y + smp
                       + [I.seed, float(res["out"][3, p]), int(res["status"][p])])
    return len(res["ids"])


def _b_values(spec: Optional[str]):
    if spec is None:
        return None
    if ":" in spec:
        lo, hi, step = (float(x) for x in spec.split(":"))
        return list(np.arange(lo, hi, step))
    return [float(x) for x in spec.split(",")]


def main(argv=None):
    ap = argparse.ArgumentParser(description="Run an input file on the GPU and write CSV output.")
    ap.add_argument("input")
    ap.add_argument("--n", type=int, default=1000, help="trajectories per impact parameter")
    ap.add_argument("--b", default=None, help="impact parameters: lo:hi:step or a,b,c "
                                              "(default: the file's b)")
    ap.add_argument("--short", default=None, help="short CSV (appended)")
    ap.add_argument("--long", default=None, help="long CSV (appended)")
    ap.add_argument("--rk", type=int, default=None, help="0: DOPRI5 (default), 1: DOP853")
    ap.add_argument("--levels", default="bs", choices=["bs", "dvr"],
                    help="internal energies: Bohr-Sommerfeld or the file's DVR grid")
    ap.add_argument("--device", type=int, default=0)
    a = ap.parse_args(argv)
    calc = load_input(a.input)
    res = run(calc, a.n, _b_values(a.b), device=a.device, rk=a.rk, levels=a.levels)
    if a.short:
        write_short(a.short, res)
    if a.long:
        write_long(a.long, res)
    tot = res["xs"][:, Q.XS_COUNTS:Q.XS_COUNTS + 6].sum(axis=0)
    print(json.dumps({"seed": calc.seed, "seed_from_file": calc.seed_from_file,
                      "trajectories": int(len(res["ids"])),
                      "counts [q, r1, r2, d, unresolved, failed]": [int(x) for x in tot]}))


if __name__ == "__main__":
    main()
