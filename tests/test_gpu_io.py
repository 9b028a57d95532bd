"""GPU run of an input file in the paper's JSON layout through the CSV
outputs: counts, per-trajectory rows and draws consistent with the run and
with the oracle's initial conditions for the same file."""
import csv
import json

import numpy as np
import pytest

import qcams_workloads as W
from paper_2304_02731_amd import qcams_io as IO
from test_io import _listing1_input

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


def test_input_file_run_and_csv(torch, orc, tmp_path):
    from paper_2304_02731_amd import qcams as Q
    path = tmp_path / "inputs.json"
    path.write_text(json.dumps(_listing1_input(seed=12345)))
    calc = IO.load_input(str(path))
    res = IO.run(calc, 96, [0.0, 1.0, 2.0])
    n = len(res["ids"])
    assert n == 288 and np.all(res["status"] != Q.RUNNING)
    short, long_ = str(tmp_path / "short.csv"), str(tmp_path / "long.csv")
    IO.write_short(short, res)
    IO.write_long(long_, res)
    srows = list(csv.DictReader(open(short)))
    assert [float(r["b"]) for r in srows] == [0.0, 1.0, 2.0]
    lrows = list(csv.DictReader(open(long_)))
    assert len(lrows) == n
    for k, r in enumerate(srows):
        mine = [x for x in lrows if float(x["b"]) == float(r["b"])]
        assert int(r["N"]) == len(mine) == 96
        for key, col in (("N_q", "n_q"), ("N_r1", "n_r1"), ("N_r2", "n_r2"), ("N_d", "n_d")):
            assert int(r[key]) == sum(int(x[col]) for x in mine)
    # the run's draws are the oracle's for the same file
    sys = orc.make_system(calc.system, masses_me=calc.system.masses_me)
    prm = orc.make_params(calc.params)
    for p in (0, 100, 287):
        I = res["instances"][p // 96]
        lev = orc.level(sys, I.v, I.j)
        _, _, smp = orc.init(sys, prm, orc.make_instance(I), lev, int(res["ids"][p]))
        assert np.array_equal(res["sample"][:5, p], smp[:5])
        assert float(lrows[p]["cos_theta"]) == smp[1] and float(lrows[p]["chi"]) == smp[4]
    # the command line
    IO.main([str(path), "--n", "32", "--b", "0:1:0.5", "--short", str(tmp_path / "cli.csv")])
    rows = list(csv.DictReader(open(tmp_path / "cli.csv")))
    assert [float(r["b"]) for r in rows] == [0.0, 0.5] and all(int(r["N"]) == 32 for r in rows)
