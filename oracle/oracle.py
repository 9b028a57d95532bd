"""ctypes wrapper of the C oracle (qcams_oracle.c) plus the aggregate step
(cross sections, Gaussian-binning distributions) in plain numpy.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Sequence

import numpy as np

import qcams_workloads as W

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qcams_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, strict IEEE double (no fast-math,
    no FMA contraction), one shared object next to the source."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Pair(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("m", C.c_int32), ("pad", C.c_int32),
                ("p", C.c_double * 6)]


class System(C.Structure):
    _fields_ = [("mass", C.c_double * 3), ("pair", Pair * 3)]


class Params(C.Structure):
    _fields_ = [("R0", C.c_double), ("t_stop", C.c_double), ("r_stop", C.c_double),
                ("atol", C.c_double), ("rtol", C.c_double), ("gb_sigma", C.c_double),
                ("h_fixed", C.c_double), ("fixed_step", C.c_int32),
                ("literal_bound", C.c_int32), ("max_steps", C.c_int64), ("rk", C.c_int32),
                ("pad", C.c_int32)]


class Instance(C.Structure):
    _fields_ = [("Ec_K", C.c_double), ("b", C.c_double), ("bmax", C.c_double),
                ("b_mode", C.c_int32), ("v", C.c_int32), ("j", C.c_int32), ("pad", C.c_int32),
                ("n_traj", C.c_int64), ("first_id", C.c_int64), ("seed", C.c_uint64)]


class Record(C.Structure):
    _fields_ = [("y", C.c_double * 12), ("t", C.c_double), ("tmax", C.c_double),
                ("rstop", C.c_double), ("e0", C.c_double), ("escale", C.c_double),
                ("h", C.c_double), ("sample", C.c_double * 6), ("vprime", C.c_double),
                ("jprime", C.c_double), ("wgb", C.c_double), ("dE_rel", C.c_double),
                ("nstep", C.c_int64), ("nrej", C.c_int64), ("status", C.c_int32),
                ("label", C.c_int32), ("vt", C.c_int32), ("jt", C.c_int32)]


RECORD_DTYPE = np.dtype([("y", "<f8", 12), ("t", "<f8"), ("tmax", "<f8"), ("rstop", "<f8"),
                         ("e0", "<f8"), ("escale", "<f8"), ("h", "<f8"), ("sample", "<f8", 6),
                         ("vprime", "<f8"), ("jprime", "<f8"), ("wgb", "<f8"),
                         ("dE_rel", "<f8"), ("nstep", "<i8"), ("nrej", "<i8"),
                         ("status", "<i4"), ("label", "<i4"), ("vt", "<i4"), ("jt", "<i4")])
assert RECORD_DTYPE.itemsize == C.sizeof(Record)

_lib = None
_dp = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        L.orc_amu_in_me.restype = C.c_double
        L.orc_kelvin_in_hartree.restype = C.c_double
        L.orc_potential.argtypes = [C.POINTER(Pair), C.c_double, _dp, _dp]
        L.orc_inner_limit.argtypes = [C.POINTER(Pair)]
        L.orc_inner_limit.restype = C.c_double
        L.orc_veff_extrema.argtypes = [C.POINTER(Pair), C.c_double, C.c_double, _dp, _dp,
                                       C.POINTER(C.c_int)]
        L.orc_turning_points.argtypes = [C.POINTER(Pair), C.c_double, C.c_double, C.c_double,
                                         C.c_double, C.c_double, _dp, _dp]
        L.orc_gauss_legendre.argtypes = [C.c_int, _dp, _dp]
        for f in (L.orc_action, L.orc_period):
            f.argtypes = [C.POINTER(Pair), C.c_double, C.c_double, C.c_double, C.c_double,
                          C.c_double]
            f.restype = C.c_double
        L.orc_hamiltonian.argtypes = [C.POINTER(System), _dp]
        L.orc_hamiltonian.restype = C.c_double
        L.orc_rhs.argtypes = [C.POINTER(System), _dp, _dp]
        L.orc_level_pair.argtypes = [C.POINTER(Pair), C.c_double, C.c_int, C.c_int, _dp]
        L.orc_level.argtypes = [C.POINTER(System), C.c_int, C.c_int, _dp]
        L.orc_philox4x64_10.argtypes = [C.POINTER(C.c_uint64)] * 3
        L.orc_uniforms.argtypes = [C.c_uint64, C.c_int64, _dp]
        L.orc_init.argtypes = [C.POINTER(System), C.POINTER(Params), C.POINTER(Instance), _dp,
                               C.c_int64, _dp, _dp, _dp]
        L.orc_init_q.argtypes = [C.POINTER(System), C.POINTER(Params), C.POINTER(Instance), _dp,
                                 C.c_int64, _dp, _dp, _dp, _dp]
        L.orc_dopri5_tableau.argtypes = [_dp, _dp, _dp, _dp]
        L.orc_propagate_log.argtypes = [C.POINTER(System), C.POINTER(Params), _dp, _dp,
                                        C.POINTER(C.c_int64), C.POINTER(C.c_int64), _dp,
                                        C.c_int64, C.POINTER(C.c_int64)]
        L.orc_trial_error.argtypes = [C.POINTER(System), C.POINTER(Params), _dp, C.c_double]
        L.orc_trial_error.restype = C.c_double
        L.orc_pair_bound.argtypes = [C.POINTER(Pair), C.c_double, C.c_double, C.c_double,
                                     C.c_double, C.c_int, _dp, _dp]
        L.orc_gb_weight.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_int)]
        L.orc_gb_weight.restype = C.c_double
        L.orc_classify.argtypes = [C.POINTER(System), C.POINTER(Params), _dp] + \
            [C.POINTER(C.c_int)] * 3 + [_dp] * 5
        L.orc_run_one.argtypes = [C.POINTER(System), C.POINTER(Params), C.POINTER(Instance),
                                  _dp, C.c_int64, C.POINTER(Record), _dp]
        L.orc_run_batch.argtypes = [C.POINTER(System), C.POINTER(Params), C.POINTER(Instance),
                                    _dp, C.POINTER(C.c_int64), C.c_int64, C.c_void_p, _dp]
        L.orc_set_dop853.argtypes = [_dp] * 5
        _install_dop853(L)
        _lib = L
    return _lib


def dop853_tableau():
    """The published Dormand-Prince 8(5,3) coefficients, as tabulated by scipy."""
    from scipy.integrate._ivp import dop853_coefficients as D
    n = D.N_STAGES
    return (np.ascontiguousarray(D.A[:n, :n], dtype=np.float64), np.asarray(D.B, dtype=np.float64),
            np.asarray(D.C[:n], dtype=np.float64), np.asarray(D.E3, dtype=np.float64),
            np.asarray(D.E5, dtype=np.float64))


def _install_dop853(L):
    A, B, Cc, E3, E5 = dop853_tableau()
    arrs = [np.ascontiguousarray(a) for a in (A.ravel(), B, Cc, E3, E5)]
    L.orc_set_dop853(*[a.ctypes.data_as(_dp) for a in arrs])


def _arr(x, n=None):
    a = np.ascontiguousarray(x, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


# ----------------------------------------------------------------------------
# conversions of the workload descriptions (oracle's own)
# ----------------------------------------------------------------------------
AMU = 1822.888486209            # m_u / m_e (CODATA 2018)
KELVIN = 3.1668115634556e-6     # k_B in hartree per kelvin (CODATA 2018)
KINDS = {"morse": 0, "lj": 1, "buck": 2}


def make_pair(p: W.Pair, mu: float | None = None) -> Pair:
    """The oracle's pair.  A Morse pair given by its harmonic frequency w_e
    (the paper's input keys de, re, we) gets alpha = w_e sqrt(mu / (2 De))
    with mu the pair's reduced mass (READING: the paper names the keys, not
    the conversion; this is the harmonic limit of the Morse oscillator)."""
    q = Pair()
    q.kind = KINDS[p.kind]
    P = p.params
    if p.kind == "morse":
        if "alpha" in P:
            vals = [P["De"], P["re"], P["alpha"]]
        else:
            vals = [P["De"], P["re"], P["we"] * math.sqrt(mu / (2.0 * P["De"]))]
    elif p.kind == "lj":
        n, m = int(P["n"]), int(P["m"])
        q.n, q.m = n, m
        if "Cn" in P:
            vals = [P["Cn"], P["Cm"]]
        else:
            # V = eps[(m/(n-m))(rm/r)^n - (n/(n-m))(rm/r)^m]: depth eps at rm
            eps, rm = P["eps"], P["rm"]
            vals = [eps * m * rm ** n / (n - m), eps * n * rm ** m / (n - m)]
    else:
        vals = [P["A"], P["b"], P["C6"]]
    for i, v in enumerate(vals):
        q.p[i] = float(v)
    return q


def make_system(s: W.System, masses_me: Sequence[float] | None = None) -> System:
    out = System()
    m = masses_me if masses_me is not None else [x * AMU for x in s.masses_amu]
    for i in range(3):
        out.mass[i] = float(m[i])
        ma, mb = float(m[i]), float(m[(i + 1) % 3])        # pair AB, BC, CA
        out.pair[i] = make_pair(s.pairs[i], ma * mb / (ma + mb))
    return out


def make_params(p: W.Params) -> Params:
    q = Params()
    for f, _ in Params._fields_:
        if f != "pad":
            setattr(q, f, getattr(p, f))
    return q


def make_instance(i: W.Instance) -> Instance:
    q = Instance()
    q.Ec_K, q.b, q.bmax = i.Ec_K, i.b, i.bmax
    q.b_mode, q.v, q.j = i.b_mode, i.v, i.j
    q.n_traj, q.first_id, q.seed = i.n_traj, i.first_id, i.seed
    return q


# ----------------------------------------------------------------------------
# thin call wrappers
# ----------------------------------------------------------------------------
def potential(pair: Pair, r: float):
    V, dV = C.c_double(), C.c_double()
    lib().orc_potential(C.byref(pair), r, C.byref(V), C.byref(dV))
    return V.value, dV.value


def inner_limit(pair: Pair) -> float:
    return lib().orc_inner_limit(C.byref(pair))


def veff_extrema(pair: Pair, mu: float, J2: float):
    rw, r0, hb = C.c_double(), C.c_double(), C.c_int()
    ok = lib().orc_veff_extrema(C.byref(pair), mu, J2, C.byref(rw), C.byref(r0), C.byref(hb))
    return bool(ok), rw.value, r0.value, bool(hb.value)


def turning_points(pair, mu, J2, E, rw, r0):
    rm, rp = C.c_double(), C.c_double()
    rc = lib().orc_turning_points(C.byref(pair), mu, J2, E, rw, r0, C.byref(rm), C.byref(rp))
    return rc, rm.value, rp.value


def gauss_legendre(n: int):
    x, px = _arr(np.zeros(n))
    w, pw = _arr(np.zeros(n))
    lib().orc_gauss_legendre(n, px, pw)
    return x, w


def action(pair, mu, J2, E, rm, rp):
    return lib().orc_action(C.byref(pair), mu, J2, E, rm, rp)


def period(pair, mu, J2, E, rm, rp):
    return lib().orc_period(C.byref(pair), mu, J2, E, rm, rp)


def level_pair(pair: Pair, mu: float, v: int, j: int):
    out, p = _arr(np.zeros(4))
    rc = lib().orc_level_pair(C.byref(pair), mu, v, j, p)
    return rc, out


def level(sys: System, v: int, j: int):
    out, p = _arr(np.zeros(4))
    rc = lib().orc_level(C.byref(sys), v, j, p)
    if rc != 0:
        raise ValueError("oracle level (v=%d, j=%d) failed: %d" % (v, j, rc))
    return out


def philox4x64_10(ctr, key):
    c = (C.c_uint64 * 4)(*[int(x) for x in ctr])
    k = (C.c_uint64 * 2)(*[int(x) for x in key])
    o = (C.c_uint64 * 4)()
    lib().orc_philox4x64_10(c, k, o)
    return [int(x) for x in o]


def uniforms(seed: int, traj_id: int):
    out, p = _arr(np.zeros(6))
    lib().orc_uniforms(seed, traj_id, p)
    return out


def hamiltonian(sys: System, y) -> float:
    a, p = _arr(y)
    return lib().orc_hamiltonian(C.byref(sys), p)


def rhs(sys: System, y):
    a, p = _arr(y)
    f, pf = _arr(np.zeros(12))
    lib().orc_rhs(C.byref(sys), p, pf)
    return f


def dopri5_tableau():
    c, pc = _arr(np.zeros(7))
    a, pa = _arr(np.zeros(49))
    b, pb = _arr(np.zeros(7))
    bh, pbh = _arr(np.zeros(7))
    lib().orc_dopri5_tableau(pc, pa, pb, pbh)
    return c, a.reshape(7, 7), b, bh


def init(sys: System, prm: Params, inst: Instance, lev, traj_id: int, prop_q=None):
    lv, pl = _arr(lev)
    y, py = _arr(np.zeros(12))
    aux, pa = _arr(np.zeros(6))
    smp, ps = _arr(np.zeros(6))
    q, pq = _arr(prop_q) if prop_q is not None else (None, None)
    rc = lib().orc_init_q(C.byref(sys), C.byref(prm), C.byref(inst), pl, traj_id, py, pa, ps, pq)
    if rc != 0:
        raise ValueError("oracle init failed: %d" % rc)
    return y, aux, smp


def propagate(sys: System, prm: Params, y, aux):
    """Integrate in place until a stop rule fires; returns
    (status, y, aux, nstep, nrej); aux = {t, tmax, rstop_eff, e0, escale, h}."""
    y, py = _arr(np.array(y, dtype=np.float64, copy=True))
    aux, pa = _arr(np.array(aux, dtype=np.float64, copy=True))
    ns, nr = C.c_int64(0), C.c_int64(0)
    st = lib().orc_propagate(C.byref(sys), C.byref(prm), py, pa, C.byref(ns), C.byref(nr))
    return st, y, aux, ns.value, nr.value


def propagate_log(sys: System, prm: Params, y, aux, log_cap: int = 1 << 16):
    """propagate() with the record of its trials: returns (status, y, aux,
    nstep, nrej, trials) with trials [n, 16] = (t, trial step, error norm,
    accepted, the 12-component state the trial starts from) in order (the
    first log_cap of them)."""
    y, py = _arr(np.array(y, dtype=np.float64, copy=True))
    aux, pa = _arr(np.array(aux, dtype=np.float64, copy=True))
    ns, nr, nl = C.c_int64(0), C.c_int64(0), C.c_int64(0)
    log = np.zeros((log_cap, 16))
    st = lib().orc_propagate_log(C.byref(sys), C.byref(prm), py, pa, C.byref(ns), C.byref(nr),
                                 log.ctypes.data_as(C.POINTER(C.c_double)), log_cap,
                                 C.byref(nl))
    return st, y, aux, ns.value, nr.value, log[:min(nl.value, log_cap)].copy()


def trial_error(sys: System, prm: Params, y, h: float) -> float:
    """Error norm of one adaptive trial of step h from state y."""
    y, py = _arr(np.array(y, dtype=np.float64, copy=True))
    return lib().orc_trial_error(C.byref(sys), C.byref(prm), py, h)


def pair_bound(pair, mu, J2, E, r, literal=0):
    rw, r0 = C.c_double(), C.c_double()
    b = lib().orc_pair_bound(C.byref(pair), mu, J2, E, r, literal, C.byref(rw), C.byref(r0))
    return bool(b), rw.value, r0.value


def gb_weight(vprime: float, sigma: float):
    vt = C.c_int()
    w = lib().orc_gb_weight(vprime, sigma, C.byref(vt))
    return w, vt.value


def classify(sys: System, prm: Params, y):
    """Returns dict(label, vt, jt, vprime, jprime, w, E[3], J2[3])."""
    a, py = _arr(y)
    lab, vt, jt = C.c_int(), C.c_int(), C.c_int()
    vp, jp, w = C.c_double(), C.c_double(), C.c_double()
    E, pE = _arr(np.zeros(3))
    J2, pJ = _arr(np.zeros(3))
    lib().orc_classify(C.byref(sys), C.byref(prm), py, C.byref(lab), C.byref(vt), C.byref(jt),
                       C.byref(vp), C.byref(jp), C.byref(w), pE, pJ)
    return dict(label=lab.value, vt=vt.value, jt=jt.value, vprime=vp.value, jprime=jp.value,
                w=w.value, E=E, J2=J2)


def run_batch(sys: System, prm: Params, inst: Instance, lev, ids, prop_q=None) -> np.ndarray:
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    out = np.zeros(len(ids), dtype=RECORD_DTYPE)
    lv, pl = _arr(lev)
    q, pq = _arr(prop_q) if prop_q is not None else (None, None)
    rc = lib().orc_run_batch(C.byref(sys), C.byref(prm), C.byref(inst), pl,
                             ids.ctypes.data_as(C.POINTER(C.c_int64)), len(ids),
                             out.ctypes.data_as(C.c_void_p), pq)
    if rc != 0:
        raise ValueError("oracle run failed: %d" % rc)
    return out


# ----------------------------------------------------------------------------
# workload-level helpers
# ----------------------------------------------------------------------------
def reduced_masses(sys: System):
    mA, mB, mC = sys.mass[0], sys.mass[1], sys.mass[2]
    mu12 = 1.0 / (1.0 / mA + 1.0 / mB)
    mu123 = 1.0 / (1.0 / mC + 1.0 / (mA + mB))
    return mu12, mu123, (mu12, 1.0 / (1.0 / mB + 1.0 / mC), 1.0 / (1.0 / mC + 1.0 / mA))


def _run_chunk(args):
    wl_sys, wl_prm, inst, ids, prop_q, lev = args
    sys = make_system(wl_sys)
    prm = make_params(wl_prm)
    return run_batch(sys, prm, make_instance(inst), lev, ids, prop_q)


def run_workload(wl: W.Workload, ids_per_instance=None, processes: int = 1, prop_q=None):
    """Run trajectories of a workload through the oracle.  ids_per_instance:
    optional list (one per instance) of global trajectory ids to run; default
    all.  Returns (records, instance index per record)."""
    # the level of each distinct (v, j), once (instances of a grid share them)
    sys = make_system(wl.system)
    levels = {}
    for inst in wl.instances:
        if (inst.v, inst.j) not in levels:
            levels[(inst.v, inst.j)] = level(sys, inst.v, inst.j)
    jobs = []
    for k, inst in enumerate(wl.instances):
        ids = (np.arange(inst.first_id, inst.first_id + inst.n_traj, dtype=np.int64)
               if ids_per_instance is None else np.asarray(ids_per_instance[k], dtype=np.int64))
        if len(ids) == 0:
            continue
        step = max(1, (len(ids) + 4 * max(processes, 1) - 1) // (4 * max(processes, 1)))
        for s in range(0, len(ids), step):
            jobs.append((k, (wl.system, wl.params, inst, ids[s:s + step], prop_q,
                             levels[(inst.v, inst.j)])))
    if processes > 1:
        import multiprocessing as mp
        ctx = mp.get_context("fork")
        with ctx.Pool(processes) as pool:
            res = pool.map(_run_chunk, [j[1] for j in jobs])
    else:
        res = [_run_chunk(j[1]) for j in jobs]
    recs = np.concatenate(res) if res else np.zeros(0, dtype=RECORD_DTYPE)
    which = np.concatenate([np.full(len(r), j[0], dtype=np.int64) for j, r in zip(jobs, res)]) \
        if res else np.zeros(0, dtype=np.int64)
    return recs, which


# ----------------------------------------------------------------------------
# aggregate step: opacity, cross sections, rates, Gaussian-binning
# distributions (Sec. 2.3 Eq. (12)-(16); Sec. 4 Eq. (18)-(19)).
# ----------------------------------------------------------------------------
NCH = 4  # q, r1, r2, d


def cross_sections(wl: W.Workload, labels, weights, inst_index):
    """Per instance: P_x = (1/N) sum w_i 1[label_i = x] and its Monte Carlo
    error (population variance, which equals Eq. (16) when w = 1).
    READING of Eq. (18): sigma = 2 pi int P b db, so uniform-in-area sampling
    gives sigma = pi bmax^2 P with SE pi bmax^2 delta; fixed-b instances report
    the opacity only (sigma = nan).  Rate Eq. (19): k = sigma sqrt(2 E_c/mu123).
    Returns dict of arrays [n_inst, 4]: P, dP, sigma, dsigma, rate, counts[n_inst, 6]."""
    sys = make_system(wl.system)
    _, mu123, _ = reduced_masses(sys)
    n = len(wl.instances)
    P = np.zeros((n, NCH))
    dP = np.zeros((n, NCH))
    counts = np.zeros((n, 6), dtype=np.int64)
    labels = np.asarray(labels)
    weights = np.asarray(weights, dtype=np.float64)
    inst_index = np.asarray(inst_index)
    for k in range(n):
        sel = inst_index == k
        N = int(sel.sum())
        lab = labels[sel]
        w = weights[sel]
        for c in range(6):
            counts[k, c] = int((lab == c).sum())
        if N == 0:
            P[k] = np.nan
            dP[k] = np.nan
            continue
        for c in range(NCH):
            x = np.where(lab == c, w, 0.0)
            m = x.sum() / N
            var = (x * x).sum() / N - m * m
            P[k, c] = m
            dP[k, c] = math.sqrt(max(var, 0.0) / N)
    area = np.array([math.pi * i.bmax ** 2 if i.b_mode == W.B_AREA else np.nan
                     for i in wl.instances])
    sigma = P * area[:, None]
    dsigma = dP * area[:, None]
    Ec = np.array([i.Ec_K * KELVIN for i in wl.instances])
    rate = sigma * np.sqrt(2.0 * Ec / mu123)[:, None]
    return dict(P=P, dP=dP, sigma=sigma, dsigma=dsigma, rate=rate, counts=counts)


def sigma_from_grid(b, P, dP):
    """Eq. (18) on a fixed impact-parameter grid (READING: prefactor 2 pi),
    trapezoid rule in b; error from independent per-b errors."""
    b = np.asarray(b, dtype=np.float64)
    f = 2.0 * math.pi * np.asarray(P) * b
    wts = np.zeros_like(b)
    wts[1:] += 0.5 * np.diff(b)
    wts[:-1] += 0.5 * np.diff(b)
    sig = float((wts * f).sum())
    err = float(math.sqrt(((wts * 2.0 * math.pi * b * np.asarray(dP)) ** 2).sum()))
    return sig, err


def gb_distributions(wl: W.Workload, labels, vt, wgb, inst_index, vmax: int = 48):
    """Gaussian-binning vibrational distributions, Eq. (14)-(15): per instance
    and channel (q, r1, r2), H[v_t] = sum of W over that channel's products,
    and the total weight W = sum_vt (sum W_r + sum W_q) + N_d.
    Returns (H [n_inst, 3, vmax], Wtot [n_inst])."""
    n = len(wl.instances)
    H = np.zeros((n, 3, vmax))
    Wt = np.zeros(n)
    labels = np.asarray(labels)
    vt = np.asarray(vt)
    wgb = np.asarray(wgb, dtype=np.float64)
    inst_index = np.asarray(inst_index)
    for i in range(len(labels)):
        k, c = int(inst_index[i]), int(labels[i])
        if c < 3 and 0 <= vt[i] < vmax:
            H[k, c, vt[i]] += wgb[i]
        if c == W.DISS:
            Wt[k] += 1.0
    Wt += H.sum(axis=(1, 2))
    return H, Wt
