"""Seeded synthetic workloads for the QCT hot path.

This module only *describes* inputs: masses, pair-potential parameters,
collision-energy grids, rovibrational levels, impact-parameter modes, seeds and
integration settings.  It holds none of the method's arithmetic (no unit
conversion, no potential, no sampling); the HIP library binding and the CPU
oracle each turn these descriptions into their own structures.

The paper (Koots & Perez-Rios, arXiv:2304.02731) prints no dataset: its
workloads are parameter sets (Sec. 3.1 input keys, Sec. 4 example).  The
surfaces below are the H2 + Ca all-Morse surface and a mixed LJ / Morse /
Buckingham surface; integration settings follow the input example of Sec. 3.1.

Units: masses in unified atomic mass units (amu), energies in hartree,
lengths in bohr, collision energies in kelvin (the paper's input convention).
Pairs are listed in the order AB, BC, CA, with AB the initial molecule and C
the colliding atom (Sec. 3.1).
"""
from __future__ import annotations

import dataclasses
from typing import List

# Base seed: each configuration k uses BASE_SEED + k.
BASE_SEED = 230402731

# Outcome labels (product-count vector of Sec. 3.3 plus bookkeeping).
QUENCH, R1, R2, DISS, UNRESOLVED, FAILED = range(6)
LABEL_NAMES = ("quench", "r1_AC+B", "r2_BC+A", "diss", "unresolved", "failed")

# Trajectory status codes.
RUNNING, OK_RSTOP, OK_TMAX, FAIL_MAXSTEPS, FAIL_NONFINITE, FAIL_HMIN, COLLAPSE = range(7)

# impact-parameter modes
B_FIXED, B_AREA, B_PROPOSAL = 0, 1, 2
RK_DOPRI5, RK_DOP853 = 0, 1


@dataclasses.dataclass(frozen=True)
class Pair:
    kind: str            # "morse" | "lj" | "buck"
    params: dict         # morse: De, re, alpha | lj: n, m, eps, rm  (or Cn, Cm) | buck: A, b, C6


@dataclasses.dataclass(frozen=True)
class System:
    masses_amu: tuple    # (mA, mB, mC)
    pairs: tuple         # (AB, BC, CA)
    name: str = ""


@dataclasses.dataclass(frozen=True)
class Params:
    R0: float = 30.0
    t_stop: float = 15.0
    r_stop: float = 60.0
    # The tolerances of the paper's timing study (Sec. 3.4, Fig. 5): the
    # looser example values of Sec. 3.1 (1e-10 / 1e-11) violate the
    # |dE/E| < 1e-8 energy gate on the slow (1e3 K) trajectories.
    atol: float = 1e-11
    rtol: float = 1e-12
    # Gaussian-binning width: full width at half maximum 0.1 quanta.
    gb_sigma: float = 0.04246609001440095
    h_fixed: float = 0.0
    fixed_step: int = 0
    literal_bound: int = 0
    max_steps: int = 10_000_000
    # Runge-Kutta variant: 0 = Dormand-Prince 5(4) (the paper's RK45),
    # 1 = Dormand-Prince 8(5,3)
    rk: int = 0


@dataclasses.dataclass(frozen=True)
class Instance:
    Ec_K: float
    v: int
    j: int
    n_traj: int
    first_id: int
    seed: int
    b_mode: int = B_AREA
    b: float = 0.0
    bmax: float = 10.0


@dataclasses.dataclass
class Workload:
    name: str
    system: System
    params: Params
    instances: List[Instance]

    @property
    def n_traj(self) -> int:
        return sum(i.n_traj for i in self.instances)


def h2ca_system() -> System:
    """H2 + Ca, all Morse: H-H (De 0.1745, re 1.40, alpha 1.03) and two
    identical Ca-H pairs (De 0.0625, re 3.78, alpha 0.62)."""
    hh = Pair("morse", {"De": 0.1745, "re": 1.40, "alpha": 1.03})
    cah = Pair("morse", {"De": 0.0625, "re": 3.78, "alpha": 0.62})
    return System((1.008, 1.008, 40.078), (hh, cah, cah), "H2+Ca morse")


def mixed_system() -> System:
    """Mixed surface: A-B generalized LJ 12-6 (eps 0.02, rm 4.0), B-C Morse
    (De 0.05, re 3.5, alpha 0.8), C-A Buckingham (A 50, b 1.5, C6 40);
    masses 7, 23, 40 amu."""
    ab = Pair("lj", {"n": 12, "m": 6, "eps": 0.02, "rm": 4.0})
    bc = Pair("morse", {"De": 0.05, "re": 3.5, "alpha": 0.8})
    ca = Pair("buck", {"A": 50.0, "b": 1.5, "C6": 40.0})
    return System((7.0, 23.0, 40.0), (ab, bc, ca), "mixed lj/morse/buck")


def _instances(grid, per_inst, seed, bmax, b_mode=B_AREA, b=0.0):
    out, first = [], 0
    for (Ec, v, j) in grid:
        out.append(Instance(Ec, v, j, per_inst, first, seed, b_mode, b, bmax))
        first += per_inst
    return out


def config_small(n_traj: int = 500) -> Workload:
    """H2(v=0, j=0) + Ca at 1e4 K, b = 8 sqrt(U) a0, 500 trajectories."""
    seed = BASE_SEED + 1
    inst = [Instance(1.0e4, 0, 0, n_traj, 0, seed, B_AREA, 0.0, 8.0)]
    return Workload("h2ca_1e4K_v0j0_n500", h2ca_system(), Params(), inst)


def ec_grid_batched():
    """16 log-spaced collision energies 1e3..1e5 K."""
    return [1.0e3 * 10.0 ** (2.0 * k / 15.0) for k in range(16)]


def config_batched(per_inst: int = 1042) -> Workload:
    """16 log-spaced E_col in 1e3..1e5 K x v in {0,2,4} x j in {0,5}, b by
    area to 10 a0: 96 instances x 1042 = 100,032 trajectories."""
    seed = BASE_SEED + 2
    grid = [(Ec, v, j) for Ec in ec_grid_batched() for v in (0, 2, 4) for j in (0, 5)]
    return Workload("h2ca_batched_96inst_1e5", h2ca_system(), Params(),
                    _instances(grid, per_inst, seed, 10.0))


def config_mixed(per_inst: int = 474) -> Workload:
    """Mixed potentials: 32 log-spaced E_col 1e3..1e5 K x v 0-5 x j 0-10,
    b by area to 12 a0: 2112 instances x 474 = 1,001,088 trajectories."""
    seed = BASE_SEED + 3
    ecs = [1.0e3 * 10.0 ** (2.0 * k / 31.0) for k in range(32)]
    grid = [(Ec, v, j) for Ec in ecs for v in range(6) for j in range(11)]
    return Workload("mixed_2112inst_1e6", mixed_system(), Params(),
                    _instances(grid, per_inst, seed, 12.0))


def config_learned_train(per_inst: int = 2084) -> Workload:
    """Training set for the learned proposal: the batched instances with
    2084 trajectories each (about 2e5)."""
    w = config_batched(per_inst)
    w.name = "h2ca_learned_train_2e5"
    seed = BASE_SEED + 4
    w.instances = [dataclasses.replace(i, seed=seed) for i in w.instances]
    return w


def config_learned_target(n_traj: int = 200_000, seed_offset: int = 0) -> Workload:
    """Target of the learned proposal: dissociation of H2(v=4, j=0) + Ca at
    5e4 K, b by area to 10 a0."""
    seed = BASE_SEED + 4 + 1000 * (1 + seed_offset)
    inst = [Instance(5.0e4, 4, 0, n_traj, 0, seed, B_AREA, 0.0, 10.0)]
    return Workload("h2ca_learned_target_v4_5e4K", h2ca_system(), Params(), inst)


def config_sweep(per_inst: int = 1292) -> Workload:
    """Full sweep: 64 log-spaced E_col 1e2..1e5 K x v 0-10 x j 0-10, b by
    area to 12 a0: 7744 instances x 1292 = 10,005,248 trajectories."""
    seed = BASE_SEED + 5
    ecs = [1.0e2 * 10.0 ** (3.0 * k / 63.0) for k in range(64)]
    grid = [(Ec, v, j) for Ec in ecs for v in range(11) for j in range(11)]
    return Workload("h2ca_sweep_7744inst_1e7", h2ca_system(), Params(),
                    _instances(grid, per_inst, seed, 12.0))


def config_paper_grid(n_per_b: int = 10_000) -> Workload:
    """The paper's Sec. 4 workflow on the H2 + Ca surface: H2(v=1, j=0),
    20 fixed impact parameters 0, 0.25, ..., 4.75 a0 per collision energy."""
    seed = BASE_SEED + 6
    ecs = [1.0e4 * k for k in range(1, 11)]
    out, first = [], 0
    for Ec in ecs:
        for ib in range(20):
            out.append(Instance(Ec, 1, 0, n_per_b, first, seed, B_FIXED, 0.25 * ib, 0.0))
            first += n_per_b
    return Workload("h2ca_paper_grid_v1j0", h2ca_system(), Params(), out)


# Integration tolerances (atol, rtol): the example values of Sec. 3.1 and the
# timing-study values of Sec. 3.4 (Fig. 5).  A run uses the example values
# where its integrator keeps every trajectory of the workload inside the
# |dE/E| < 1e-8 energy gate, and the timing-study values otherwise.  Measured
# on the listed workloads (largest |dE/E| over all trajectories): DOP853 on
# the batched workload 4.8e-9 at the example values; DOPRI5 on it 2.7e-8
# (fails), DOP853 on the sweep 1.1e-7 (fails), DOP853 on the mixed surface
# 9.2e-9 (kept out: too close to the gate).
TOL_EXAMPLE = (1.0e-10, 1.0e-11)
TOL_TIMING = (1.0e-11, 1.0e-12)
EXAMPLE_TOL_KEEPS_GATE = {("h2ca_batched_96inst_1e5", RK_DOP853)}


def gated_params(wl: "Workload", rk: int) -> Params:
    """The workload's parameters with RK variant rk and the tolerances above."""
    atol, rtol = TOL_EXAMPLE if (wl.name, rk) in EXAMPLE_TOL_KEEPS_GATE else TOL_TIMING
    return dataclasses.replace(wl.params, rk=rk, atol=atol, rtol=rtol)


CONFIGS = {
    "small": config_small,
    "batched": config_batched,
    "mixed": config_mixed,
    "learned_train": config_learned_train,
    "learned_target": config_learned_target,
    "sweep": config_sweep,
    "paper_grid": config_paper_grid,
}
