"""Python binding of the QCT library (include/qcams.h): argument marshalling
only.  Every step of the path runs in the library's HIP kernels; torch
provides device memory and streams.

The library must be built (``python -m paper_2304_02731_amd.build``); there is
no fallback: every call raises if ``libqcams.so`` is missing.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import re
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqcams.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "qcams.h")

# ---- constants mirrored from include/qcams.h ----
OK, EINVAL, EUNBOUND, ENOROOT, EHIP, ENOMEM = 0, -1, -2, -3, -4, -5
MORSE, LJ, BUCK, MORSE_WE, LJ_EPS = 0, 1, 2, 3, 4
MASS_ME, MASS_AMU = 0, 1
B_FIXED, B_AREA, B_PROPOSAL = 0, 1, 2
RK_DOPRI5, RK_DOP853 = 0, 1
LEVELS_BS, LEVELS_DVR = 0, 1
MLP_NPARAM, MLP_NIN, MLP_NOUT, PROP_CELLS = 34436, 6, 4, 8192
RUNNING, OK_RSTOP, OK_TMAX, FAIL_MAXSTEPS, FAIL_NONFINITE, FAIL_HMIN, COLLAPSE = range(7)
QUENCH, R1, R2, DISS, UNRESOLVED, FAILED = range(6)
NF, NS, XS_STRIDE, VMAX, GRID_STRIDE = 18, 6, 32, 64, 24
F_X, F_P, F_T, F_TMAX, F_RSTOP, F_E0, F_ESCALE, F_H = 0, 6, 12, 13, 14, 15, 16, 17
# columns of a cross-section row
XS_N, XS_COUNTS, XS_P, XS_DP, XS_SIGMA, XS_DSIGMA, XS_RATE, XS_WTOT, XS_SUMW, XS_SUMW2 = \
    0, 1, 7, 11, 15, 19, 23, 27, 28, 29
# columns of a fixed-b grid row
G_EC, G_V, G_J, G_NB, G_BMAX, G_N, G_SIGMA, G_DSIGMA, G_RATE = 0, 1, 2, 3, 4, 5, 6, 10, 14

KIND = {"morse": MORSE, "lj": LJ, "buck": BUCK}


class QcamsError(RuntimeError):
    pass


class Pair(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("m", C.c_int32), ("pad", C.c_int32),
                ("p", C.c_double * 6)]


class System(C.Structure):
    _fields_ = [("mass", C.c_double * 3), ("pair", Pair * 3), ("mass_unit", C.c_int32),
                ("pad", C.c_int32)]


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


class StateC(C.Structure):
    _fields_ = [("d", C.c_void_p), ("nstep", C.c_void_p), ("nrej", C.c_void_p),
                ("status", C.c_void_p), ("ld", C.c_int64)]


class RunOpts(C.Structure):
    _fields_ = [("blocks", C.c_int32), ("refill_min", C.c_int32), ("check_every", C.c_int32),
                ("lpt", C.c_int32), ("graph", C.c_int32), ("rk", C.c_int32),
                ("lanes", C.c_int32), ("pad", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


class OutcomeC(C.Structure):
    _fields_ = [("label", C.c_void_p), ("vt", C.c_void_p), ("jt", C.c_void_p),
                ("d", C.c_void_p), ("ld", C.c_int64)]


_lib = None


def exported_names() -> list:
    """Function names declared in include/qcams.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qcams_[a-z_0-9]+)\s*\(", txt)))


def lib():
    """Load libqcams.so (after torch, so that both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise QcamsError("libqcams.so is not built: run python -m paper_2304_02731_amd.build")
    import torch  # noqa: F401  (loads the HIP runtime torch uses)
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.qcams_create.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(System), C.POINTER(Params)]
    L.qcams_system_resolve.argtypes = [C.POINTER(System), C.POINTER(System)]
    L.qcams_destroy.argtypes = [vp]
    L.qcams_destroy.restype = None
    L.qcams_last_error.argtypes = [vp]
    L.qcams_last_error.restype = C.c_char_p
    L.qcams_levels.argtypes = [vp, i32, vp, vp, vp]
    L.qcams_set_instances.argtypes = [vp, C.POINTER(Instance), i32]
    L.qcams_init_conditions.argtypes = [vp, vp, i64, C.POINTER(StateC), vp, vp]
    L.qcams_propagate.argtypes = [vp, C.POINTER(StateC), i64, vp]
    L.qcams_classify.argtypes = [vp, C.POINTER(StateC), i64, C.POINTER(OutcomeC), vp]
    L.qcams_cross_sections.argtypes = [vp, C.POINTER(OutcomeC), vp, vp, i64, vp, vp, vp]
    L.qcams_run.argtypes = [vp, C.POINTER(RunOpts), C.POINTER(StateC), vp, C.POINTER(OutcomeC),
                            vp, vp, vp, vp]
    L.qcams_run_noalloc.argtypes = [vp, C.POINTER(RunOpts), C.POINTER(StateC), vp,
                                    C.POINTER(OutcomeC), vp, vp, vp, vp]
    L.qcams_last_run_kernel_ms.argtypes = [vp, C.POINTER(C.c_double)]
    L.qcams_last_run_wave_steps.argtypes = [vp, C.POINTER(C.c_int64)]
    L.qcams_last_run_options.argtypes = [vp, C.POINTER(RunOpts)]
    L.qcams_grid_groups.argtypes = [vp, C.POINTER(C.c_int32), vp]
    L.qcams_dvr_levels.argtypes = [vp, i32, C.c_double, C.c_double, i32, vp, vp, vp]
    L.qcams_set_level_method.argtypes = [vp, i32, i32, C.c_double, C.c_double]
    L.qcams_propagate_record.argtypes = [vp, C.POINTER(StateC), i64, vp, i32, vp, vp]
    L.qcams_grid_cross_sections.argtypes = [vp, vp, vp, vp]
    L.qcams_autotune.argtypes = [vp, C.POINTER(StateC), C.POINTER(OutcomeC), vp, vp, i32, i32,
                                 C.c_double, C.POINTER(RunOpts), C.POINTER(C.c_double)]
    L.qcams_mlp_create.argtypes = [C.POINTER(vp), C.c_int, vp, C.c_uint64]
    L.qcams_mlp_destroy.argtypes = [vp]
    L.qcams_mlp_destroy.restype = None
    L.qcams_mlp_last_error.argtypes = [vp]
    L.qcams_mlp_last_error.restype = C.c_char_p
    L.qcams_mlp_get_params.argtypes = [vp, vp]
    L.qcams_mlp_set_params.argtypes = [vp, vp]
    L.qcams_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
    L.qcams_mlp_gradient.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp]
    L.qcams_mlp_adam.argtypes = [vp, vp, C.c_float, vp]
    L.qcams_mlp_train_epoch.argtypes = [vp, vp, vp, vp, i64, i32, C.c_float, vp, vp]
    L.qcams_mlp_features.argtypes = [vp, vp, vp, i64, C.POINTER(OutcomeC), i64, vp, vp, vp]
    L.qcams_proposal_build.argtypes = [vp, vp, i32, i32, C.c_double, vp]
    L.qcams_proposal_set.argtypes = [vp, vp]
    for name in exported_names():
        getattr(L, name)  # raises if a declared symbol is missing
    _lib = L
    return L


# ---------------------------------------------------------------------------
# marshalling of workload descriptions into the ABI structures (duck-typed:
# .masses_amu or explicit electron masses, .pairs with .kind / .params;
# params objects with the qcams_params field names).  Values are copied as
# given; the library converts units and input forms (qcams_system_resolve).
# ---------------------------------------------------------------------------
def make_pair(p) -> Pair:
    q = Pair()
    kind = p.kind if isinstance(p.kind, int) else KIND[p.kind]
    P = p.params
    if kind == MORSE:
        if "alpha" in P:
            vals = [P["De"], P["re"], P["alpha"]]
        else:                      # the paper's input form: harmonic frequency w_e
            kind = MORSE_WE
            vals = [P["De"], P["re"], P["we"]]
    elif kind == LJ:
        q.n, q.m = int(P["n"]), int(P["m"])
        if "Cn" in P:
            vals = [P["Cn"], P["Cm"]]
        else:                      # depth eps and position rm of the minimum
            kind = LJ_EPS
            vals = [P["eps"], P["rm"]]
    else:
        vals = [P["A"], P["b"], P["C6"]]
    q.kind = kind
    for i, v in enumerate(vals):
        q.p[i] = float(v)
    return q


def make_system(system, masses_me: Optional[Sequence[float]] = None) -> System:
    s = System()
    if masses_me is not None:
        m, s.mass_unit = masses_me, MASS_ME
    else:
        m, s.mass_unit = system.masses_amu, MASS_AMU
    for i in range(3):
        s.mass[i] = float(m[i])
        s.pair[i] = make_pair(system.pairs[i])
    return s


def resolve_system(system, masses_me: Optional[Sequence[float]] = None) -> System:
    """The system in the library's canonical form (qcams_system_resolve):
    electron masses, Morse / LJ / Buckingham parameters.  Needs no GPU."""
    s = make_system(system, masses_me)
    out = System()
    rc = lib().qcams_system_resolve(C.byref(s), C.byref(out))
    if rc != OK:
        raise QcamsError("qcams_system_resolve failed (%d): %s"
                         % (rc, lib().qcams_last_error(None).decode()))
    return out


def make_params(p) -> Params:
    q = Params()
    for f, _ in Params._fields_:
        if f != "pad":
            setattr(q, f, getattr(p, f, 0))
    return q


def make_instances(instances) -> C.Array:
    arr = (Instance * len(instances))()
    for k, i in enumerate(instances):
        a = arr[k]
        a.Ec_K, a.b, a.bmax = i.Ec_K, i.b, i.bmax
        a.b_mode, a.v, a.j = i.b_mode, i.v, i.j
        a.n_traj, a.first_id, a.seed = i.n_traj, i.first_id, i.seed
    return arr


# ---------------------------------------------------------------------------
# device buffers (torch tensors)
# ---------------------------------------------------------------------------
@dataclass
class State:
    d: "torch.Tensor"        # float64 [NF, ld]
    nstep: "torch.Tensor"    # int32 [ld]
    nrej: "torch.Tensor"     # int32 [ld]
    status: "torch.Tensor"   # uint8 [ld]

    @property
    def ld(self) -> int:
        return self.d.shape[1]

    def c(self) -> StateC:
        return StateC(self.d.data_ptr(), self.nstep.data_ptr(), self.nrej.data_ptr(),
                      self.status.data_ptr(), self.ld)


@dataclass
class Outcome:
    label: "torch.Tensor"    # uint8 [ld]
    vt: "torch.Tensor"       # int16 [ld]
    jt: "torch.Tensor"       # int16 [ld]
    d: "torch.Tensor"        # float64 [4, ld]: v', j', W, dE/E

    @property
    def ld(self) -> int:
        return self.d.shape[1]

    def c(self) -> OutcomeC:
        return OutcomeC(self.label.data_ptr(), self.vt.data_ptr(), self.jt.data_ptr(),
                        self.d.data_ptr(), self.ld)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Context:
    """One system + parameter set on one GPU (qcams_ctx)."""

    def __init__(self, system, params, device: int = 0, masses_me=None):
        import torch
        self.device = device
        self.torch_device = torch.device("cuda", device)
        L = lib()
        self._sys = make_system(system, masses_me)
        self._prm = make_params(params)
        h = C.c_void_p()
        with torch.cuda.device(device):
            rc = L.qcams_create(C.byref(h), device, C.byref(self._sys), C.byref(self._prm))
        if rc != OK:
            raise QcamsError("qcams_create failed (%d): %s" % (rc, L.qcams_last_error(None).decode()))
        self._h = h
        self.instances = []

    def close(self):
        if getattr(self, "_h", None):
            lib().qcams_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != OK:
            raise QcamsError("%s failed (%d): %s" % (what, rc, lib().qcams_last_error(self._h).decode()))

    # ---- synchronous set-up ----
    def dvr_levels(self, npts: int, xmin: float, xmax: float, v: Sequence[int],
                   j: Sequence[int]) -> np.ndarray:
        """(E, r-, r+, tau) per (v, j) from the Colbert-Miller DVR (qcams_dvr_levels)."""
        v = np.ascontiguousarray(v, dtype=np.int32)
        j = np.ascontiguousarray(j, dtype=np.int32)
        out = np.zeros((len(v), 4))
        self._check(lib().qcams_dvr_levels(self._h, npts, xmin, xmax, len(v), v.ctypes.data,
                                           j.ctypes.data, out.ctypes.data), "qcams_dvr_levels")
        return out

    def set_level_method(self, method: int, npts: int = 0, xmin: float = 0.0,
                         xmax: float = 0.0):
        """Levels of later set_instances calls: LEVELS_BS or LEVELS_DVR with a grid."""
        self._check(lib().qcams_set_level_method(self._h, method, npts, xmin, xmax),
                    "qcams_set_level_method")

    def levels(self, v: Sequence[int], j: Sequence[int]) -> np.ndarray:
        v = np.ascontiguousarray(v, dtype=np.int32)
        j = np.ascontiguousarray(j, dtype=np.int32)
        out = np.zeros((len(v), 4))
        self._check(lib().qcams_levels(self._h, len(v), v.ctypes.data, j.ctypes.data,
                                       out.ctypes.data), "qcams_levels")
        return out

    def set_instances(self, instances):
        arr = make_instances(instances)
        self._check(lib().qcams_set_instances(self._h, arr, len(instances)), "qcams_set_instances")
        self.instances = list(instances)

    # ---- buffers ----
    def new_state(self, n: int) -> State:
        import torch
        dev = self.torch_device
        return State(torch.zeros((NF, n), dtype=torch.float64, device=dev),
                     torch.zeros(n, dtype=torch.int32, device=dev),
                     torch.zeros(n, dtype=torch.int32, device=dev),
                     torch.zeros(n, dtype=torch.uint8, device=dev))

    def new_outcome(self, n: int) -> Outcome:
        import torch
        dev = self.torch_device
        return Outcome(torch.zeros(n, dtype=torch.uint8, device=dev),
                       torch.zeros(n, dtype=torch.int16, device=dev),
                       torch.zeros(n, dtype=torch.int16, device=dev),
                       torch.zeros((4, n), dtype=torch.float64, device=dev))

    # ---- asynchronous path ----
    def init_conditions(self, ids, state: State, sample=None, stream=None):
        n = ids.numel()
        sp = sample.data_ptr() if sample is not None else None
        self._check(lib().qcams_init_conditions(self._h, ids.data_ptr(), n, C.byref(state.c()),
                                                sp, _stream(stream)), "qcams_init_conditions")

    def propagate(self, state: State, n: Optional[int] = None, stream=None):
        n = state.ld if n is None else n
        self._check(lib().qcams_propagate(self._h, C.byref(state.c()), n, _stream(stream)),
                    "qcams_propagate")

    def classify(self, state: State, outcome: Outcome, n: Optional[int] = None, stream=None):
        n = state.ld if n is None else n
        self._check(lib().qcams_classify(self._h, C.byref(state.c()), n, C.byref(outcome.c()),
                                         _stream(stream)), "qcams_classify")

    def cross_sections(self, outcome: Outcome, ids, weight=None, n: Optional[int] = None,
                       with_hist: bool = True, stream=None):
        import torch
        n = ids.numel() if n is None else n
        xs = torch.zeros((len(self.instances), XS_STRIDE), dtype=torch.float64,
                         device=self.torch_device)
        hist = torch.zeros((len(self.instances), 3, VMAX), dtype=torch.float64,
                           device=self.torch_device) if with_hist else None
        self._check(lib().qcams_cross_sections(
            self._h, C.byref(outcome.c()), ids.data_ptr(),
            weight.data_ptr() if weight is not None else None, n, xs.data_ptr(),
            hist.data_ptr() if hist is not None else None, _stream(stream)),
            "qcams_cross_sections")
        return xs, hist

    @property
    def n_total(self) -> int:
        return sum(i.n_traj for i in self.instances)

    def new_run_buffers(self):
        """Buffers for qcams_run sized to the installed instances."""
        import torch
        n = self.n_total
        dev = self.torch_device
        return dict(state=self.new_state(n), outcome=self.new_outcome(n),
                    sample=torch.zeros((NS, n), dtype=torch.float64, device=dev),
                    ids=torch.zeros(n, dtype=torch.int64, device=dev),
                    xs=torch.zeros((len(self.instances), XS_STRIDE), dtype=torch.float64, device=dev),
                    hist=torch.zeros((len(self.instances), 3, VMAX), dtype=torch.float64, device=dev))

    def run(self, buf, opts: Optional[RunOpts] = None, stream=None, with_sample=True,
            with_hist=True):
        """Fused persistent run of every installed trajectory (qcams_run)."""
        st, out = buf["state"], buf["outcome"]
        self._check(lib().qcams_run(
            self._h, C.byref(opts) if opts is not None else None, C.byref(st.c()),
            buf["sample"].data_ptr() if with_sample else None, C.byref(out.c()),
            buf["ids"].data_ptr(), buf["xs"].data_ptr(),
            buf["hist"].data_ptr() if with_hist else None, _stream(stream)), "qcams_run")
        return buf["xs"], buf["hist"]

    def run_noalloc(self, buf, opts: Optional[RunOpts] = None, stream=None, with_sample=True,
                    with_hist=True):
        """qcams_run_noalloc: the fused run with its work buffers in the
        library's static device scratch (no allocation in the call)."""
        st, out = buf["state"], buf["outcome"]
        self._check(lib().qcams_run_noalloc(
            self._h, C.byref(opts) if opts is not None else None, C.byref(st.c()),
            buf["sample"].data_ptr() if with_sample else None, C.byref(out.c()),
            buf["ids"].data_ptr(), buf["xs"].data_ptr(),
            buf["hist"].data_ptr() if with_hist else None, _stream(stream)), "qcams_run_noalloc")
        return buf["xs"], buf["hist"]

    def last_run_kernel_ms(self) -> float:
        """Duration of the persistent kernel of the last run (HIP events)."""
        ms = C.c_double()
        self._check(lib().qcams_last_run_kernel_ms(self._h, C.byref(ms)), "qcams_last_run_kernel_ms")
        return ms.value

    def last_run_wave_steps(self) -> int:
        """Trial-step loop iterations the persistent waves of the last run
        executed with at least one slot stepping."""
        v = C.c_int64()
        self._check(lib().qcams_last_run_wave_steps(self._h, C.byref(v)), "qcams_last_run_wave_steps")
        return v.value

    def propagate_record(self, st: State, rec_max: int, n: Optional[int] = None, stream=None):
        """qcams_propagate recording (t, r_AB, r_BC, r_CA) after every accepted
        step: returns (rec [n, rec_max, 4], counts [n]) device tensors."""
        import torch
        n = st.d.shape[1] if n is None else n
        rec = torch.zeros((n, rec_max, 4), dtype=torch.float64, device=self.torch_device)
        cnt = torch.zeros(n, dtype=torch.int32, device=self.torch_device)
        self._check(lib().qcams_propagate_record(self._h, C.byref(st.c()), n, rec.data_ptr(),
                                                 rec_max, cnt.data_ptr(), _stream(stream)),
                    "qcams_propagate_record")
        return rec, cnt

    def grid_groups(self):
        """(number of fixed-b groups, group index of every instance)."""
        import numpy as np
        ng = C.c_int32()
        g = np.zeros(len(self.instances), dtype=np.int32)
        self._check(lib().qcams_grid_groups(self._h, C.byref(ng), g.ctypes.data), "qcams_grid_groups")
        return ng.value, g

    def grid_cross_sections(self, xs, stream=None):
        """Per-group sigma, error and rate on fixed-b grids (qcams_grid_cross_sections)."""
        import torch
        ng, _ = self.grid_groups()
        out = torch.zeros((max(ng, 1), GRID_STRIDE), dtype=torch.float64, device=self.torch_device)
        self._check(lib().qcams_grid_cross_sections(self._h, xs.data_ptr(), out.data_ptr(),
                                                    _stream(stream)),
                    "qcams_grid_cross_sections")
        return out[:ng]

    def last_run_options(self) -> RunOpts:
        """Effective options of the last run (qcams_last_run_options)."""
        o = RunOpts()
        self._check(lib().qcams_last_run_options(self._h, C.byref(o)), "qcams_last_run_options")
        return o

    def autotune(self, buf, reps: int = 1, search_rk: bool = False, energy_gate: float = 1e-8,
                 retune: bool = False):
        """Fastest qcams_run options on the installed instances (qcams_autotune);
        with search_rk also the RK variant, among those keeping the energy gate.
        A result cached for the same key is returned unless retune is set."""
        if retune:
            reps = -max(1, reps)
        best = RunOpts()
        ms = C.c_double()
        self._check(lib().qcams_autotune(self._h, C.byref(buf["state"].c()),
                                         C.byref(buf["outcome"].c()), buf["ids"].data_ptr(),
                                         buf["xs"].data_ptr(), reps, int(search_rk),
                                         float(energy_gate), C.byref(best), C.byref(ms)),
                    "qcams_autotune")
        return best, ms.value

    # ---- learned proposal ----
    def mlp_features(self, ids, sample, outcome: Outcome, n: Optional[int] = None, stream=None):
        """Network inputs x [n, 6] (float32) and labels y [n] (int32, -1 = not a
        class) of classified trajectories."""
        import torch
        n = ids.numel() if n is None else n
        x = torch.zeros((n, MLP_NIN), dtype=torch.float32, device=self.torch_device)
        y = torch.zeros(n, dtype=torch.int32, device=self.torch_device)
        self._check(lib().qcams_mlp_features(self._h, ids.data_ptr(), sample.data_ptr(),
                                             sample.shape[1], C.byref(outcome.c()), n,
                                             x.data_ptr(), y.data_ptr(), _stream(stream)),
                    "qcams_mlp_features")
        return x, y

    def proposal_build(self, mlp, inst: int, channel: int, alpha: float):
        """Build and install the proposal of instance `inst` for `channel`;
        returns the cell probabilities q [PROP_CELLS] (float64, device)."""
        import torch
        q = torch.zeros(PROP_CELLS, dtype=torch.float64, device=self.torch_device)
        self._check(lib().qcams_proposal_build(self._h, mlp._h if mlp is not None else None, inst,
                                               channel, alpha, q.data_ptr()), "qcams_proposal_build")
        return q

    def proposal_set(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        assert q.shape == (PROP_CELLS,)
        self._check(lib().qcams_proposal_set(self._h, q.ctypes.data), "qcams_proposal_set")

    def all_ids(self):
        import torch
        ids = [torch.arange(i.first_id, i.first_id + i.n_traj, dtype=torch.int64)
               for i in self.instances]
        return torch.cat(ids).to(self.torch_device)


class MLP:
    """The proposal network (qcams_mlp): 6 -> 128 -> 128 -> 128 -> 4."""

    def __init__(self, params=None, seed: int = 0, device: int = 0):
        import torch
        self.torch_device = torch.device("cuda", device)
        L = lib()
        h = C.c_void_p()
        p = None
        if params is not None:
            self._init = np.ascontiguousarray(params, dtype=np.float32)
            assert self._init.shape == (MLP_NPARAM,)
            p = self._init.ctypes.data
        with torch.cuda.device(device):
            rc = L.qcams_mlp_create(C.byref(h), device, p, seed)
        if rc != OK:
            raise QcamsError("qcams_mlp_create failed (%d): %s" % (rc, L.qcams_mlp_last_error(None).decode()))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().qcams_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != OK:
            raise QcamsError("%s failed (%d): %s" % (what, rc, lib().qcams_mlp_last_error(self._h).decode()))

    def params(self) -> np.ndarray:
        out = np.zeros(MLP_NPARAM, dtype=np.float32)
        self._check(lib().qcams_mlp_get_params(self._h, out.ctypes.data), "qcams_mlp_get_params")
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._check(lib().qcams_mlp_set_params(self._h, p.ctypes.data), "qcams_mlp_set_params")

    def forward(self, x, stream=None):
        import torch
        n = x.shape[0]
        prob = torch.zeros((n, MLP_NOUT), dtype=torch.float32, device=self.torch_device)
        self._check(lib().qcams_mlp_forward(self._h, x.data_ptr(), n, prob.data_ptr(), _stream(stream)),
                    "qcams_mlp_forward")
        return prob

    def gradient(self, x, y, idx=None, n: Optional[int] = None, stream=None):
        import torch
        n = (idx.numel() if idx is not None else x.shape[0]) if n is None else n
        g = torch.zeros(MLP_NPARAM, dtype=torch.float32, device=self.torch_device)
        loss = torch.zeros(1, dtype=torch.float32, device=self.torch_device)
        self._check(lib().qcams_mlp_gradient(self._h, x.data_ptr(), y.data_ptr(),
                                             idx.data_ptr() if idx is not None else None, n,
                                             g.data_ptr(), loss.data_ptr(), _stream(stream)),
                    "qcams_mlp_gradient")
        return g, loss

    def adam(self, grad, lr: float, stream=None):
        self._check(lib().qcams_mlp_adam(self._h, grad.data_ptr(), lr, _stream(stream)), "qcams_mlp_adam")

    def train_epoch(self, x, y, perm, batch: int, lr: float, loss_sum, stream=None):
        self._check(lib().qcams_mlp_train_epoch(self._h, x.data_ptr(), y.data_ptr(), perm.data_ptr(),
                                                perm.numel(), batch, lr, loss_sum.data_ptr(),
                                                _stream(stream)), "qcams_mlp_train_epoch")
