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
    """The oracle timed on a bounded stratified sample (here one id of every
    100th of the small workload's 500 trajectories, one process)."""
    import qcams_workloads as W
    B = _bench()
    wl = W.config_small(n_traj=500)
    wl.params = W.gated_params(wl, W.RK_DOP853)
    cb = B.cpu_baseline(wl, 100, 1)
    assert set(cb) == {"value", "unit", "cores", "kind", "sample"}
    assert cb["kind"] == "oracle" and cb["unit"] == "trajectories/s" and cb["cores"] == 1
    assert cb["value"] > 0 and "5 trajectories" in cb["sample"]
    json.dumps(cb)


def test_roofline_tables_cover_every_workload_and_variant():
    B = _bench()
    for surface in set(s for s, _ in B.WORKLOADS.values()):
        assert surface in B.KINDS
        for rk in B.RK_NAMES.values():
            assert B.F_STEP[(surface, rk)] > 0
    # a DOP853 step does more work than a DOPRI5 step on the same surface
    for surface in ("morse", "mixed"):
        assert B.F_STEP[(surface, 1)] > 2 * B.F_STEP[(surface, 0)]
    for (wl, kernel), nbytes in B.TRAFFIC.items():
        assert wl in B.WORKLOADS and kernel.startswith("k_persistent<") and nbytes > 0
    assert B.PEAK_FP64_VECTOR == 78.6e12
