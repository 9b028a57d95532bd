"""Pins of the oracle's Dormand-Prince 8(5,3) variant: one step equals
scipy's Runge-Kutta step with the same published tableau; order 8 by step
halving on the periodic two-body orbit (Eq. (7)); adaptive runs agree with
scipy's DOP853 integrator; energy conservation on full trajectories."""
import dataclasses
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.integrate._ivp import rk as RK

import qcams_workloads as W


def _params(**kw):
    return dataclasses.replace(W.Params(), rk=1, **kw)


def test_tableau_consistency(orc):
    A, B, C, E3, E5 = orc.dop853_tableau()
    assert np.allclose(A.sum(axis=1), C, atol=1e-15)
    assert abs(B.sum() - 1.0) < 1e-15
    # the error combinations annihilate constants (both embedded methods are consistent)
    assert abs(E5.sum()) < 1e-15 and abs(E3.sum()) < 1e-15
    # quadrature conditions of order 8 for b: sum b_i c_i^(k-1) = 1/k
    for k in range(1, 9):
        assert abs((B * C ** (k - 1)).sum() - 1.0 / k) < 1e-14, k


def test_one_step_matches_scipy(orc):
    sys = orc.make_system(W.h2ca_system())
    A, B, C, E3, E5 = orc.dop853_tableau()
    wl = W.config_batched()
    I = wl.instances[60]
    lev = orc.level(sys, I.v, I.j)
    y0, aux, _ = orc.init(sys, orc.make_params(wl.params), orc.make_instance(I), lev, I.first_id)
    h = 3.0
    f = lambda t, y: orc.rhs(sys, y)
    K = np.zeros((13, 12))
    ys, fs = RK.rk_step(f, 0.0, y0, f(0, y0), h, A, B, C, K)
    prm = orc.make_params(_params(fixed_step=1, h_fixed=h))
    st, y1, a1, ns, nr = orc.propagate(sys, prm, y0, np.r_[0.0, h, 1e9, 0, 1, 0.0])
    assert ns == 1
    assert np.allclose(y1, ys, rtol=1e-14, atol=1e-15)


def _two_body(orc, v=0):
    hh = W.Pair("morse", {"De": 0.1745, "re": 1.40, "alpha": 1.03})
    zero = W.Pair("morse", {"De": 0.0, "re": 3.78, "alpha": 0.62})
    sys = orc.make_system(W.System((1.008, 1.008, 40.078), (hh, zero, zero)))
    lev = orc.level(sys, v, 0)
    y0 = np.zeros(12)
    y0[2] = lev[2]
    y0[5] = -1000.0
    return sys, lev, y0


def test_order_eight(orc):
    """Full-state error at non-symmetric times against a 512-step reference:
    halving the step divides it by 2^8.  (The reference's own truncation
    error is ~(24/512)^8 of the 24-step error; a finer reference would add
    more rounding than it removes: at 4096 steps its accumulated rounding,
    ~5e-13, is as large as the 24-step error.)"""
    sys, lev, y0 = _two_body(orc, 2)
    for frac in (0.36, 0.37, 0.38):
        T = frac * lev[3]

        def run(n):
            prm = orc.make_params(_params(fixed_step=1, h_fixed=T / n))
            return orc.propagate(sys, prm, y0, np.r_[0.0, T, 1e9, 0, 1, 0.0])[1]

        ref = run(512)
        errs = [np.abs(run(n) - ref).max() for n in (6, 12, 24)]
        r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
        assert 200 < r1 < 330 and 200 < r2 < 330, (frac, r1, r2)


def test_adaptive_agrees_with_scipy_dop853(orc):
    wl = W.config_batched()
    sys = orc.make_system(wl.system)
    prm = orc.make_params(_params())
    I = wl.instances[60]
    lev = orc.level(sys, I.v, I.j)
    f = lambda t, y: orc.rhs(sys, y)
    for tid in range(3):
        y0, aux, _ = orc.init(sys, prm, orc.make_instance(I), lev, I.first_id + tid)
        T = 3 * lev[3]
        st, y1, a1, ns, nr = orc.propagate(sys, prm, y0, np.r_[0.0, T, 1e9, 0, 1, 0.0])
        sol = solve_ivp(f, (0, T), y0, method="DOP853", rtol=1e-13, atol=1e-13)
        scale = np.maximum(np.abs(sol.y[:, -1]), 1.0)
        assert np.all(np.abs(y1 - sol.y[:, -1]) / scale < 1e-9)


@pytest.mark.slow
def test_energy_conservation_dop853(orc):
    wl = W.config_batched()
    sys = orc.make_system(wl.system)
    prm = orc.make_params(_params())
    for k in (8, 47, 95):
        I = wl.instances[k]
        lev = orc.level(sys, I.v, I.j)
        recs = orc.run_batch(sys, prm, orc.make_instance(I), lev, np.arange(I.first_id, I.first_id + 6))
        assert np.all(np.abs(recs["dE_rel"]) < 1e-8), np.abs(recs["dE_rel"]).max()
        assert np.all(recs["label"] != W.FAILED)
