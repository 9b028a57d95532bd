"""Pins of the oracle's equations of motion and integrator: Hamilton's
equations in Jacobi coordinates (Eq. (2)-(4)) against Newton's equations of
the Cartesian Hamiltonian (Eq. (1)); exactness on free flight; the
two-body vibrational period (Eq. (7)); order 5 of the Runge-Kutta pair;
energy / angular-momentum conservation; time reversal; scipy's RK45."""
import dataclasses
import math
from fractions import Fraction as F

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import qcams_workloads as W


# ---------------------------------------------------------------------------
# an independent Cartesian formulation (Eq. (1)), numpy, Morse pairs only
# ---------------------------------------------------------------------------
def _cart(sys_w, orc):
    m = np.array(sys_w.masses_amu) * orc.AMU
    pairs = [(0, 1), (1, 2), (2, 0)]
    par = [(p.params["De"], p.params["re"], p.params["alpha"]) for p in sys_w.pairs]

    def V(x):  # x: [3 atoms, 3]
        tot = 0.0
        for (i, k), (De, re, a) in zip(pairs, par):
            r = np.linalg.norm(x[k] - x[i])
            tot += De * (1 - math.exp(-a * (r - re))) ** 2 - De
        return tot

    def forces(x):
        f = np.zeros((3, 3))
        for (i, k), (De, re, a) in zip(pairs, par):
            d = x[k] - x[i]
            r = np.linalg.norm(d)
            e = math.exp(-a * (r - re))
            dV = 2 * De * a * e * (1 - e)
            f[k] -= dV * d / r
            f[i] += dV * d / r
        return f

    def to_cart(y):
        mA, mB, mC = m
        M = m.sum()
        r1, r2, p1, p2 = y[0:3], y[3:6], y[6:9], y[9:12]
        cA, cB = mA / (mA + mB), mB / (mA + mB)
        Rab = -(mC / M) * r2           # centre of mass at the origin
        x = np.array([Rab - cB * r1, Rab + cA * r1, Rab + r2])
        mu12 = mA * mB / (mA + mB)
        mu123 = mC * (mA + mB) / M
        v1, v2 = p1 / mu12, p2 / mu123
        Vab = -(mC / M) * v2
        vel = np.array([Vab - cB * v1, Vab + cA * v1, Vab + v2])
        return x, vel

    def jacobi_rhs(y):
        mA, mB, mC = m
        M = m.sum()
        mu12 = mA * mB / (mA + mB)
        mu123 = mC * (mA + mB) / M
        x, vel = to_cart(y)
        f = forces(x)
        acc = f / m[:, None]
        dp1 = mu12 * (acc[1] - acc[0])
        dp2 = mu123 * (acc[2] - (m[0] * acc[0] + m[1] * acc[1]) / (mA + mB))
        return np.concatenate([y[6:9] / mu12, y[9:12] / mu123, dp1, dp2])

    def energy(y):
        x, vel = to_cart(y)
        return 0.5 * (m[:, None] * vel ** 2).sum() + V(x)

    return jacobi_rhs, energy


def _random_state(rng):
    return np.concatenate([rng.normal(0, 1.5, 3) + [0.3, 0.2, 1.2],
                           rng.normal(0, 2.0, 3) + [0, 1.0, -4.0],
                           rng.normal(0, 3.0, 3), rng.normal(0, 5.0, 3)])


def test_rhs_and_energy_match_cartesian_newton(orc):
    sw = W.h2ca_system()
    sys = orc.make_system(sw)
    jr, en = _cart(sw, orc)
    rng = np.random.default_rng(1)
    for _ in range(20):
        y = _random_state(rng)
        f = orc.rhs(sys, y)
        g = jr(y)
        assert np.allclose(f, g, rtol=1e-11, atol=1e-13 * np.abs(g).max())
        assert orc.hamiltonian(sys, y) == pytest.approx(en(y), rel=1e-12, abs=1e-14)


def test_rhs_unequal_masses_and_pairs(orc):
    """Different masses and three different Morse pairs expose any swapped
    mass ratio or pair index in the chain rule."""
    sw = W.System((1.008, 2.014, 40.078),
                  (W.Pair("morse", {"De": 0.1745, "re": 1.40, "alpha": 1.03}),
                   W.Pair("morse", {"De": 0.05, "re": 3.5, "alpha": 0.8}),
                   W.Pair("morse", {"De": 0.0625, "re": 3.78, "alpha": 0.62})))
    sys = orc.make_system(sw)
    jr, en = _cart(sw, orc)
    rng = np.random.default_rng(2)
    for _ in range(20):
        y = _random_state(rng)
        f = orc.rhs(sys, y)
        g = jr(y)
        assert np.allclose(f, g, rtol=1e-11, atol=1e-13 * np.abs(g).max())
        assert orc.hamiltonian(sys, y) == pytest.approx(en(y), rel=1e-12, abs=1e-14)


def test_rhs_is_gradient_of_hamiltonian(orc):
    """dP/dt = -dH/drho and drho/dt = dH/dP by finite differences, for all
    three potential kinds (mixed surface)."""
    sys = orc.make_system(W.mixed_system())
    rng = np.random.default_rng(3)
    for _ in range(10):
        y = _random_state(rng) * 0.6 + np.r_[0, 0, 3.5, 0, 0, -6.0, np.zeros(6)]
        f = orc.rhs(sys, y)
        for i in range(12):
            h = 1e-6 * max(1.0, abs(y[i]))
            yp, ym = y.copy(), y.copy()
            yp[i] += h
            ym[i] -= h
            d = (orc.hamiltonian(sys, yp) - orc.hamiltonian(sys, ym)) / (2 * h)
            expect = d if i >= 6 else -d
            k = i - 6 if i >= 6 else i + 6
            assert f[k] == pytest.approx(expect, rel=1e-6, abs=1e-9)


def test_tableau_order_conditions(orc):
    """Dormand-Prince 5(4): b satisfies the order conditions through order 5,
    bhat through order 4 (not 5); row sums of A equal c."""
    c, A, b, bh = orc.dopri5_tableau()
    Af = [[F(x).limit_denominator(10 ** 7) for x in row] for row in A]
    cf = [F(x).limit_denominator(10 ** 7) for x in c]
    for i in range(7):
        assert abs(sum(A[i]) - c[i]) < 1e-15
    def conds(w):
        w = [F(x).limit_denominator(10 ** 7) for x in w]
        s = range(7)
        Ac = [sum(Af[i][k] * cf[k] for k in s) for i in s]
        Ac2 = [sum(Af[i][k] * cf[k] ** 2 for k in s) for i in s]
        AAc = [sum(Af[i][k] * Ac[k] for k in s) for i in s]
        Ac3 = [sum(Af[i][k] * cf[k] ** 3 for k in s) for i in s]
        AcAc = [sum(Af[i][k] * cf[k] * Ac[k] for k in s) for i in s]
        AAc2 = [sum(Af[i][k] * Ac2[k] for k in s) for i in s]
        AAAc = [sum(Af[i][k] * AAc[k] for k in s) for i in s]
        out = {
            1: [sum(w) - 1],
            2: [sum(w[i] * cf[i] for i in s) - F(1, 2)],
            3: [sum(w[i] * cf[i] ** 2 for i in s) - F(1, 3), sum(w[i] * Ac[i] for i in s) - F(1, 6)],
            4: [sum(w[i] * cf[i] ** 3 for i in s) - F(1, 4),
                sum(w[i] * cf[i] * Ac[i] for i in s) - F(1, 8),
                sum(w[i] * Ac2[i] for i in s) - F(1, 12),
                sum(w[i] * AAc[i] for i in s) - F(1, 24)],
            5: [sum(w[i] * cf[i] ** 4 for i in s) - F(1, 5),
                sum(w[i] * cf[i] ** 2 * Ac[i] for i in s) - F(1, 10),
                sum(w[i] * Ac[i] ** 2 for i in s) - F(1, 20),
                sum(w[i] * cf[i] * Ac2[i] for i in s) - F(1, 15),
                sum(w[i] * cf[i] * AAc[i] for i in s) - F(1, 30),
                sum(w[i] * Ac3[i] for i in s) - F(1, 20),
                sum(w[i] * AcAc[i] for i in s) - F(1, 40),
                sum(w[i] * AAc2[i] for i in s) - F(1, 60),
                sum(w[i] * AAAc[i] for i in s) - F(1, 120)],
        }
        return out
    cb = conds(b)
    for order in range(1, 6):
        assert all(abs(float(x)) < 1e-12 for x in cb[order]), order
    ch = conds(bh)
    for order in range(1, 5):
        assert all(abs(float(x)) < 1e-12 for x in ch[order]), order
    assert any(abs(float(x)) > 1e-6 for x in ch[5])
    # FSAL: the last stage is evaluated at the 5th-order solution
    assert np.allclose(A[6, :6], b[:6]) and b[6] == 0.0


def _params(**kw):
    return dataclasses.replace(W.Params(), **kw)


def test_free_flight_is_exact(orc):
    """With every potential switched off the motion is uniform; any RK method
    integrates it exactly (to rounding)."""
    zero = W.Pair("morse", {"De": 0.0, "re": 1.4, "alpha": 1.0})
    sw = W.System((1.008, 1.008, 40.078), (zero, zero, zero))
    sys = orc.make_system(sw)
    mu12, mu123, _ = orc.reduced_masses(sys)
    y0 = np.r_[0.3, -0.2, 1.1, 0.5, 2.0, -30.0, 1.5, 0.7, -0.4, 0.2, -0.1, 12.0]
    aux = np.r_[0.0, 3000.0, 1e9, 0.0, 1.0, 0.0]
    st, y, aux2, ns, nr = orc.propagate(sys, orc.make_params(_params()), y0, aux)
    assert st == W.OK_TMAX and aux2[0] == 3000.0
    expect = y0.copy()
    expect[0:3] += y0[6:9] / mu12 * 3000.0
    expect[3:6] += y0[9:12] / mu123 * 3000.0
    assert np.allclose(y, expect, rtol=1e-13, atol=1e-12)


def _two_body(orc, v=0):
    """AB Morse molecule with the atom far away and its pairs switched off."""
    hh = W.Pair("morse", {"De": 0.1745, "re": 1.40, "alpha": 1.03})
    zero = W.Pair("morse", {"De": 0.0, "re": 3.78, "alpha": 0.62})
    sw = W.System((1.008, 1.008, 40.078), (hh, zero, zero))
    sys = orc.make_system(sw)
    lev = orc.level(sys, v, 0)
    y0 = np.zeros(12)
    y0[2] = lev[2]            # at rest at the outer turning point
    y0[5] = -1000.0
    return sys, lev, y0


def test_two_body_period(orc):
    """Eq. (7): a vibrating molecule alone returns to its outer turning point
    after tau_v, conserving its energy."""
    sys, lev, y0 = _two_body(orc, 2)
    tau = lev[3]
    aux = np.r_[0.0, tau, 1e9, 0.0, 1.0, 0.0]
    st, y, aux2, ns, nr = orc.propagate(sys, orc.make_params(_params()), y0, aux)
    assert st == W.OK_TMAX
    assert y[2] == pytest.approx(lev[2], rel=1e-9)
    assert abs(y[8]) < 1e-7
    assert orc.hamiltonian(sys, y) == pytest.approx(orc.hamiltonian(sys, y0), rel=1e-11)


def test_fixed_step_convergence_order(orc):
    """Step halving on the periodic two-body orbit: the error after one period
    falls by 2^5 per halving (DOPRI5 is 5th order)."""
    sys, lev, y0 = _two_body(orc, 0)
    tau = lev[3]
    errs = []
    for n in (100, 200, 400):
        prm = orc.make_params(_params(fixed_step=1, h_fixed=tau / n))
        aux = np.r_[0.0, tau, 1e9, 0.0, 1.0, 0.0]
        st, y, aux2, ns, nr = orc.propagate(sys, prm, y0, aux)
        assert ns in (n, n + 1)  # a rounding-sized last step may be added
        # the bond length at the turning point is insensitive (to 2nd order) to
        # the small quadrature error of tau, so it measures the RK error alone
        errs.append(abs(y[2] - y0[2]))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 26.0 < r1 < 38.0 and 26.0 < r2 < 38.0


def _run_ids(orc, wl, k, ids):
    sys = orc.make_system(wl.system)
    prm = orc.make_params(wl.params)
    I = wl.instances[k]
    lev = orc.level(sys, I.v, I.j)
    return orc.run_batch(sys, prm, orc.make_instance(I), lev, ids), sys


@pytest.mark.slow
def test_energy_and_angular_momentum_conservation(orc):
    """|dE|/E_scale < 1e-8 per trajectory (energy gate) and conserved total
    angular momentum rho1 x P1 + rho2 x P2, on full trajectories."""
    wl = W.config_batched()
    for k in (8, 47, 95):      # 1e3 K (v=4 j=5), ~1e4 K (v=4 j=5), 1e5 K (v=4 j=5)
        I = wl.instances[k]
        recs, sys = _run_ids(orc, wl, k, np.arange(I.first_id, I.first_id + 6))
        assert np.all(np.abs(recs["dE_rel"]) < 1e-8)
        # angular momentum: recompute the initial state from the same id
        lev = orc.level(sys, I.v, I.j)
        for t, r in zip(range(I.first_id, I.first_id + 6), recs):
            y0, _, _ = orc.init(sys, orc.make_params(wl.params), orc.make_instance(I), lev, t)
            L0 = np.cross(y0[0:3], y0[6:9]) + np.cross(y0[3:6], y0[9:12])
            y = r["y"]
            L1 = np.cross(y[0:3], y[6:9]) + np.cross(y[3:6], y[9:12])
            assert np.allclose(L1, L0, rtol=0, atol=1e-6 * max(1.0, np.linalg.norm(L0)))


def test_time_reversal(orc):
    """Integrate forward over about two vibrational periods of the collision,
    flip the momenta and integrate back: the start is recovered to the
    integrator's tolerance."""
    wl = W.config_batched()
    sys = orc.make_system(wl.system)
    prm = orc.make_params(wl.params)
    I = wl.instances[47]
    lev = orc.level(sys, I.v, I.j)
    y0, aux0, _ = orc.init(sys, prm, orc.make_instance(I), lev, I.first_id + 3)
    T = 2 * lev[3]
    aux = np.r_[0.0, T, 1e9, aux0[3], aux0[4], 0.0]
    st, y1, a1, _, _ = orc.propagate(sys, prm, y0, aux)
    assert st == W.OK_TMAX
    yb = y1.copy()
    yb[6:] *= -1
    st, y2, a2, _, _ = orc.propagate(sys, prm, yb, np.r_[0.0, T, 1e9, aux0[3], aux0[4], 0.0])
    y2[6:] *= -1
    scale = np.maximum(np.abs(y0), 1.0)
    assert np.all(np.abs(y2 - y0) / scale < 1e3 * wl.params.rtol * 100)


def test_agrees_with_scipy_rk45_short_horizon(orc):
    """scipy's RK45 (the paper's integrator) on the independent Cartesian RHS
    and the oracle agree over a short horizon at tight tolerance."""
    wl = W.config_batched()
    sys = orc.make_system(wl.system)
    prm = orc.make_params(wl.params)
    I = wl.instances[60]
    lev = orc.level(sys, I.v, I.j)
    jr, en = _cart(wl.system, orc)
    for tid in range(3):
        y0, aux0, _ = orc.init(sys, prm, orc.make_instance(I), lev, I.first_id + tid)
        T = 3 * lev[3]
        st, y1, _, _, _ = orc.propagate(sys, prm, y0, np.r_[0.0, T, 1e9, 0, 1, 0.0])
        sol = solve_ivp(lambda t, y: jr(y), (0, T), y0, method="RK45", rtol=1e-12,
                        atol=1e-13)
        yr = sol.y[:, -1]
        scale = np.maximum(np.abs(yr), 1.0)
        assert np.all(np.abs(y1 - yr) / scale < 1e-8)


def test_stop_rules(orc):
    """r_stop: the run ends on the first accepted step with a pair beyond
    r_stop_eff; max_steps ends it with a failure status."""
    wl = W.config_batched()
    sys = orc.make_system(wl.system)
    I = wl.instances[90]
    lev = orc.level(sys, I.v, I.j)
    prm = orc.make_params(wl.params)
    y0, aux0, _ = orc.init(sys, prm, orc.make_instance(I), lev, I.first_id)
    st, y, aux, ns, nr = orc.propagate(sys, prm, y0, aux0)
    assert st == W.OK_RSTOP
    r1, r2 = y[0:3], y[3:6]
    cA = cB = 0.5
    d = max(np.linalg.norm(r1), np.linalg.norm(r2 - cA * r1), np.linalg.norm(-r2 - cB * r1))
    assert d > aux0[2]
    prm2 = orc.make_params(_params(max_steps=7))
    st, y, aux, ns, nr = orc.propagate(sys, prm2, y0, aux0)
    assert st == W.FAIL_MAXSTEPS and ns == 7
