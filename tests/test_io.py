"""Input files in the paper's JSON layout (Sec. 3.1, Listing 1) and the
short / long CSV outputs (Sec. 3.3): host-side logic, no GPU."""
import csv
import json
import math
import os

import numpy as np
import pytest

import qcams_workloads as W
from paper_2304_02731_amd import qcams_io as IO
from paper_2304_02731_amd import qcams as Q

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "listing1_inputs.json")


def _listing1_input(seed=None, kinds=("morse", "morse", "morse")):
    """The Listing 1 file: the paper collapses BC and CA, which carry the
    same keys as AB; here they repeat AB's values."""
    g = json.load(open(GOLDEN))
    pp = {k: dict(g["AB"], npts=1000, xmin=0.5, xmax=10) for k in ("AB", "BC", "CA")}
    return {"vi": 0, "ji": 0, "Ec (K)": 30000, "b": 0, "r0": 30, "seed": seed,
            "potential_AB": kinds[0], "potential_BC": kinds[1], "potential_CA": kinds[2],
            "masses": g["masses_me"], "int_params": g["int_params"], "potential_params": pp}


def test_load_listing1_fields():
    calc = IO.load_input(_listing1_input(seed=7))
    g = json.load(open(GOLDEN))
    assert calc.system.masses_me == (g["masses_me"]["ma"], g["masses_me"]["mb"],
                                     g["masses_me"]["mc"])
    p = calc.params
    assert (p.R0, p.t_stop, p.r_stop, p.atol, p.rtol) == (30.0, 15.0, 60.0, 1e-10, 1e-11)
    assert (calc.v, calc.j, calc.Ec_K, calc.b, calc.seed, calc.seed_from_file) == (0, 0, 30000.0, 0.0, 7, True)
    assert calc.dvr["AB"] == {"npts": 1000, "xmin": 0.5, "xmax": 10}
    assert calc.guesses["AB"] == {"re": g["AB"]["morse"]["re"]}
    # a null seed is drawn and reported
    c2 = IO.load_input(_listing1_input(seed=None))
    assert not c2.seed_from_file and 0 <= c2.seed < 2 ** 63


def test_morse_range_from_harmonic_frequency(orc):
    """alpha = w_e sqrt(mu / (2 D_e)): the oracle's Bohr-Sommerfeld levels
    (pinned to the Morse closed form) of the converted pair give the
    closed-form spacing E_1 - E_0 = w_e - w_e^2 / (2 D_e) of the file's w_e."""
    calc = IO.load_input(_listing1_input(seed=1))
    g = json.load(open(GOLDEN))["AB"]["morse"]
    sys = orc.make_system(calc.system, masses_me=calc.system.masses_me)
    e0 = orc.level(sys, 0, 0)[0]
    e1 = orc.level(sys, 1, 0)[0]
    we, de = g["we"], g["de"]
    assert e1 - e0 == pytest.approx(we - we * we / (2.0 * de), rel=1e-10)
    assert e0 == pytest.approx(0.5 * we - we * we / (16.0 * de) - de, rel=1e-10)


def test_morse_pair_goes_to_the_library_by_harmonic_frequency():
    """The binding hands the file's (de, re, we) over unchanged, as the
    library's Morse input form; the library's conversion equals the
    oracle's alpha = w_e sqrt(mu / (2 D_e)) with the pair's reduced mass."""
    import oracle as orc
    calc = IO.load_input(_listing1_input(seed=1))
    g = json.load(open(GOLDEN))["AB"]["morse"]
    q = Q.make_pair(calc.system.pairs[0])
    assert (q.kind, q.p[0], q.p[1], q.p[2]) == (Q.MORSE_WE, g["de"], g["re"], g["we"])
    r = Q.resolve_system(calc.system, masses_me=calc.system.masses_me)
    o = orc.make_system(calc.system, masses_me=calc.system.masses_me)
    for i in range(3):
        assert r.pair[i].kind == Q.MORSE
        assert r.pair[i].p[2] == pytest.approx(o.pair[i].p[2], rel=1e-15)


def test_lj_and_buckingham_parameters():
    calc = IO.load_input(_listing1_input(seed=1, kinds=("lj", "buck", "morse")))
    g = json.load(open(GOLDEN))["AB"]
    lj, bk = calc.system.pairs[0], calc.system.pairs[1]
    assert lj.kind == "lj" and lj.params == {"n": 12, "m": 6, "Cn": g["lj"]["cn"], "Cm": g["lj"]["cm"]}
    assert bk.kind == "buck" and bk.params == {"A": g["buck"]["a"], "b": g["buck"]["b"],
                                               "C6": g["buck"]["c6"]}
    q = Q.make_pair(lj)
    assert (q.kind, q.n, q.m, q.p[0], q.p[1]) == (Q.LJ, 12, 6, g["lj"]["cn"], g["lj"]["cm"])
    with pytest.raises(ValueError):
        IO._pair("harmonic", {})


def _fake_result():
    inst = [W.Instance(2e4, 1, 0, 3, 0, 11, W.B_FIXED, 0.0, 0.0),
            W.Instance(2e4, 1, 0, 3, 3, 11, W.B_FIXED, 0.5, 0.0)]
    n = 6
    xs = np.zeros((2, Q.XS_STRIDE))
    label = np.array([0, 3, 1, 0, 0, 4], dtype=np.uint8)
    for k in range(2):
        xs[k, Q.XS_N] = 3
        for c in label[3 * k:3 * k + 3]:
            xs[k, Q.XS_COUNTS + c] += 1
    state = np.arange(18 * n, dtype=np.float64).reshape(18, n)
    out = np.vstack([np.linspace(0, 1, n), np.zeros(n), np.full(n, 0.25), np.full(n, 1e-12)])
    sample = np.vstack([np.zeros(n), np.full(n, 0.1), np.full(n, 0.2), np.full(n, 0.3),
                        np.full(n, 0.4), np.ones(n)])
    return {"instances": inst, "xs": xs, "ids": np.arange(n), "state": state,
            "status": np.full(n, 1, dtype=np.uint8), "label": label,
            "vt": np.array([1, 0, 2, 1, 0, 0], dtype=np.int16),
            "jt": np.array([3, 0, 5, 1, 2, 0], dtype=np.int16), "out": out, "sample": sample}


def test_short_and_long_csv(tmp_path):
    res = _fake_result()
    short, long_ = str(tmp_path / "s.csv"), str(tmp_path / "l.csv")
    assert IO.write_short(short, res) == 2
    assert IO.write_short(short, res) == 2          # appends without a second header
    rows = list(csv.reader(open(short)))
    assert rows[0] == IO.SHORT_COLUMNS and len(rows) == 5
    assert rows[1][:9] == ["20000.0", "0.0", "3", "1", "1", "0", "1", "0", "0"]
    assert rows[2][:9] == ["20000.0", "0.5", "3", "2", "0", "0", "0", "1", "0"]
    assert IO.write_long(long_, res, append=False) == 6
    rows = list(csv.DictReader(open(long_)))
    assert len(rows) == 6
    for p, r in enumerate(rows):
        lab = int(res["label"][p])
        assert [int(r[k]) for k in ("n_q", "n_r1", "n_r2", "n_d")] == [int(lab == c) for c in range(4)]
        if lab < 3:
            assert (int(r["v_t"]), float(r["w"]), int(r["j_t"])) == (res["vt"][p], 0.25, res["jt"][p])
        else:   # dissociation (and unresolved): s_f = (0, 0, 0)
            assert (int(r["v_t"]), float(r["w"]), int(r["j_t"])) == (0, 0.0, 0)
        assert float(r["rho1_x"]) == res["state"][0, p] and float(r["t_f"]) == res["state"][12, p]
        assert float(r["P2_z"]) == res["state"][11, p]
        assert float(r["cos_theta"]) == 0.1 and float(r["chi"]) == 0.4
        assert int(r["seed"]) == 11 and float(r["b"]) == (0.0 if p < 3 else 0.5)


def test_b_values_spec():
    assert IO._b_values("0:5:0.25") == list(np.arange(0, 5, 0.25))
    assert IO._b_values("0,1.5,2") == [0.0, 1.5, 2.0]
    assert IO._b_values(None) is None
