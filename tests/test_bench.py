"""CPU tests of the benchmark's contract: the one-GPU rule, the CPU-oracle
baseline leg and the tables the roofline is computed from."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_without_gpu_the_bench_refuses_rather_than_falls_back():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--no-cpu-baseline"],
                       capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 2
    assert "needs a GPU" in r.stderr
    assert not any(l.startswith("{") for l in r.stdout.splitlines())


def test_cpu_baseline_leg_reports_the_contract_keys():
    """The oracle timed on bounded systematic samples (here every 100th of
    the small workload's 500 trajectories in a one-process pool, and every
    250th on one core)."""
    import qcams_workloads as W
    B = _bench()
    wl = W.config_small(n_traj=500)
    wl.params = W.gated_params(wl, W.RK_DOP853)
    cb = B.cpu_baseline(wl, 100, 250, 1)
    assert set(cb) == {"value", "unit", "cores", "kind", "sample", "one_core"}
    assert cb["kind"] == "oracle" and cb["unit"] == "trajectories/s" and cb["cores"] == 1
    assert cb["value"] > 0 and "5 trajectories" in cb["sample"]
    one = cb["one_core"]
    assert one["trajectories_per_s"] > 0 and one["trial_steps_per_s"] > 0
    assert one["ms_per_trajectory"] == pytest.approx(1e3 / one["trajectories_per_s"])
    assert "2 trajectories" in one["sample"]
    json.dumps(cb)


def test_roofline_tables_cover_every_workload_and_variant():
    """Every workload's surface has FP64 work per trial step for both RK
    variants: the hand count from the step function's source agrees with the
    hardware counters within 3 %, and the method-only count (exponential,
    square root and reciprocal as one operation each) is below it."""
    import qcams_workloads as W
    B = _bench()
    for surface in set(v[0] for v in B.WORKLOADS.values()):
        assert surface in B.KINDS
        for rk in B.RK_NAMES.values():
            f = B.F_STEP[(surface, rk)]
            assert 0 < f["method"] < f["hand"]
            assert abs(f["hand"] / f["counter"] - 1.0) < 0.03, (surface, rk, f)
    # a DOP853 step does more work than a DOPRI5 step on the same surface
    for surface in ("morse", "mixed"):
        assert B.F_STEP[(surface, 1)]["hand"] > 2 * B.F_STEP[(surface, 0)]["hand"]
    names = {W.CONFIGS[k]().name for k in B.WORKLOADS}
    for (wl, kernel), nbytes in B.TRAFFIC.items():
        assert wl in names and kernel.startswith("k_persistent<") and nbytes > 0
    assert B.PEAK_FP64_VECTOR == 78.6e12


def test_oracle_sample_strides_over_all_trajectories():
    """The sample takes every k-th trajectory counted across instances: one
    id per k overall, spread over the instances in order."""
    import numpy as np
    import qcams_workloads as W
    B = _bench()
    wl = W.config_batched(per_inst=7)
    per = B._oracle_sample(wl, 5)
    ids = np.concatenate(per)
    assert np.array_equal(ids, np.arange(0, wl.n_traj, 5))
    for i, p in zip(wl.instances, per):
        assert np.all((p >= i.first_id) & (p < i.first_id + i.n_traj))


def test_outcomes_by_status_counts():
    import numpy as np
    B = _bench()
    lab = np.array([0, 0, 4, 4, 4, 5, 3], dtype=np.uint8)
    st = np.array([1, 2, 1, 2, 2, 3, 1], dtype=np.uint8)
    o = B.outcomes_by_status(np, lab, st)
    assert o == {"quench": {"ok_rstop": 1, "ok_tmax": 1}, "diss": {"ok_rstop": 1},
                 "unresolved": {"ok_rstop": 1, "ok_tmax": 2}, "failed": {"fail_maxsteps": 1}}
