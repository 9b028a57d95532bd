"""Pins of the oracle's potentials, units, quadrature and Bohr-Sommerfeld
levels against closed forms, the paper's printed inputs and independent
library routines (numpy, scipy)."""
import json
import warnings
import math
import os

import numpy as np
import pytest
from scipy import integrate, optimize

import qcams_workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")


def _morse(De, re, a):
    return W.Pair("morse", {"De": De, "re": re, "alpha": a})


def test_mass_unit_matches_listing1(orc):
    # Sec. 3.1, Listing 1 gives the hydrogen mass as 1837.47165336 m_e (1.008 amu).
    g = json.load(open(os.path.join(GOLD, "listing1_inputs.json")))
    amu = orc.lib().orc_amu_in_me()
    assert amu == pytest.approx(orc.AMU, rel=0, abs=0)
    assert 1.008 * amu == pytest.approx(g["masses_me"]["ma"], rel=5e-8)


@pytest.mark.parametrize("kind,par,rs", [
    ("morse", {"De": 0.1745, "re": 1.4, "alpha": 1.03}, [0.6, 1.4, 2.3, 7.0]),
    ("lj", {"n": 12, "m": 6, "eps": 0.02, "rm": 4.0}, [3.2, 4.0, 6.5, 11.0]),
    ("lj", {"n": 9, "m": 4, "Cn": 3.0e3, "Cm": 60.0}, [1.5, 2.5, 4.0]),
    ("buck", {"A": 50.0, "b": 1.5, "C6": 40.0}, [2.0, 3.0, 9.9, 15.0]),
])
def test_derivative_is_derivative(orc, kind, par, rs):
    p = orc.make_pair(W.Pair(kind, par))
    for r in rs:
        h = 1e-5 * r
        Vp, _ = orc.potential(p, r + h)
        Vm, _ = orc.potential(p, r - h)
        Vp2, _ = orc.potential(p, r + 2 * h)
        Vm2, _ = orc.potential(p, r - 2 * h)
        fd = (8 * (Vp - Vm) - (Vp2 - Vm2)) / (12 * h)
        _, dV = orc.potential(p, r)
        assert dV == pytest.approx(fd, rel=1e-7, abs=1e-12)


def test_morse_shape(orc):
    p = orc.make_pair(_morse(0.1745, 1.4, 1.03))
    V, dV = orc.potential(p, 1.4)
    assert V == -0.1745 and dV == 0.0
    V, _ = orc.potential(p, 60.0)
    assert abs(V) < 1e-20


def test_lj_convention_pinned_by_listing1(orc):
    """READING of the LJ sign (Sec. 3.2): with V = Cn/r^n - Cm/r^m the 12-6
    well depth Cm^2/(4 Cn) reproduces the Morse depth printed in the same
    listing (de = 0.16456603489)."""
    g = json.load(open(os.path.join(GOLD, "listing1_inputs.json")))["AB"]
    lj = g["lj"]
    p = orc.make_pair(W.Pair("lj", {"n": lj["n"], "m": lj["m"], "Cn": lj["cn"], "Cm": lj["cm"]}))
    ok, rw, r0, hb = orc.veff_extrema(p, 918.7, 0.0)
    assert ok and not hb
    V, _ = orc.potential(p, rw)
    assert -V == pytest.approx(g["morse"]["de"], rel=1e-10)
    # the swapped (printed) form would have no well at all
    assert rw == pytest.approx((2 * lj["cn"] / lj["cm"]) ** (1 / 6), rel=1e-12)


def test_lj_from_eps_rm(orc):
    p = orc.make_pair(W.Pair("lj", {"n": 12, "m": 6, "eps": 0.02, "rm": 4.0}))
    assert p.p[0] == pytest.approx(335544.32, rel=1e-14)
    assert p.p[1] == pytest.approx(163.84, rel=1e-14)
    V, dV = orc.potential(p, 4.0)
    assert V == pytest.approx(-0.02, rel=1e-13) and abs(dV) < 1e-15


def test_buckingham_inner_maximum(orc):
    """Sec. 3.2: a Buckingham potential has a short-range maximum and collapses
    inside it; the oracle's inner limit is that maximum (V' = 0, V'' < 0)."""
    A, b, C6 = 50.0, 1.5, 40.0
    p = orc.make_pair(W.Pair("buck", {"A": A, "b": b, "C6": C6}))
    rb = orc.inner_limit(p)
    ref = optimize.brentq(lambda r: -A * b * math.exp(-b * r) + 6 * C6 / r ** 7, 0.5, 3.0,
                          xtol=1e-15, rtol=1e-15)
    assert rb == pytest.approx(ref, rel=1e-12)
    _, d1 = orc.potential(p, rb * 0.99)
    _, d2 = orc.potential(p, rb * 1.01)
    assert d1 > 0 > d2


@pytest.mark.parametrize("n", [8, 64, 256])
def test_gauss_legendre_vs_numpy(orc, n):
    x, w = orc.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.allclose(x, xr, rtol=0, atol=2e-15)
    assert np.allclose(w, wr, rtol=1e-10, atol=0)
    # exact for polynomials of degree <= 2n - 1
    for k in (0, 2, n, 2 * n - 2):
        assert (w * x ** k).sum() == pytest.approx(2.0 / (k + 1), rel=1e-13, abs=1e-15)
    assert abs((w * x ** (2 * n - 1)).sum()) < 1e-14


# --- Morse j = 0: Bohr-Sommerfeld is exact -----------------------------------
def _morse_exact(De, re, a, mu, v):
    om = a * math.sqrt(2 * De / mu)
    E = -De + om * (v + 0.5) - om ** 2 * (v + 0.5) ** 2 / (4 * De)
    s = math.sqrt(1 + E / De)
    rm = re - math.log(1 + s) / a
    rp = re - math.log(1 - s) / a
    tau = 2 * math.pi / (om * math.sqrt(-E / De))
    return E, rm, rp, tau


@pytest.mark.parametrize("pair,mu_amu", [((0.1745, 1.40, 1.03), (1.008, 1.008)),
                                         ((0.0625, 3.78, 0.62), (40.078, 1.008))])
def test_morse_levels_closed_form(orc, pair, mu_amu):
    De, re, a = pair
    p = orc.make_pair(_morse(De, re, a))
    m1, m2 = (x * orc.AMU for x in mu_amu)
    mu = m1 * m2 / (m1 + m2)
    vmax = int(math.floor(math.sqrt(2 * mu * De) / a - 0.5))
    for v in range(0, vmax + 1):
        rc, out = orc.level_pair(p, mu, v, 0)
        assert rc == 0, v
        E, rm, rp, tau = _morse_exact(De, re, a, mu, v)
        assert out[0] == pytest.approx(E, rel=5e-13, abs=1e-15)
        assert out[1] == pytest.approx(rm, rel=1e-11)
        assert out[2] == pytest.approx(rp, rel=1e-11)
        # Eq. (7) at the oracle's own energy: the closed-form period of the
        # classical Morse oscillator, 2 pi / (omega sqrt(-E / De)).  Measured
        # within 4e-14 for every level below the top two, 2e-13 at the top.
        om = a * math.sqrt(2 * De / mu)
        tau_at_E = 2 * math.pi / (om * math.sqrt(-out[0] / De))
        assert out[3] == pytest.approx(tau_at_E, rel=1e-13 if v <= vmax - 2 else 1e-12), v
        assert out[3] == pytest.approx(tau, rel=1e-12), v
    rc, _ = orc.level_pair(p, mu, vmax + 1, 0)
    assert rc == -2  # unbound


def test_h2_printed_values(orc):
    """H2 v=0 and v=4 with the surface's Morse parameters (closed forms)."""
    s = orc.make_system(W.h2ca_system())
    out0 = orc.level(s, 0, 0)
    out4 = orc.level(s, 4, 0)
    assert out0[0] == pytest.approx(-0.164606863975204, rel=1e-12)
    assert out4[0] == pytest.approx(-0.095854426232671, rel=1e-12)
    assert out0[3] == pytest.approx(322.2545028656, rel=1e-9)


def _scipy_level(V, mu, v, j, rlo, rhi):
    """Independent Bohr-Sommerfeld solution with scipy quad/brentq."""
    J2 = j * (j + 1.0)
    Ve = lambda r: V(r) + J2 / (2 * mu * r * r)
    res = optimize.minimize_scalar(Ve, bounds=(rlo, rhi), method="bounded",
                                   options={"xatol": 1e-12})
    rw = res.x

    def tp(E):
        a = optimize.brentq(lambda r: Ve(r) - E, rlo, rw, xtol=1e-15, rtol=1e-15)
        b = optimize.brentq(lambda r: Ve(r) - E, rw, rhi, xtol=1e-15, rtol=1e-15)
        return a, b

    def act(E):
        a, b = tp(E)
        val, _ = integrate.quad(lambda r: math.sqrt(max(E - Ve(r), 0.0)), a, b,
                                epsabs=0, epsrel=1e-13, limit=400)
        return math.sqrt(2 * mu) / math.pi * val

    E = optimize.brentq(lambda E: act(E) - (v + 0.5), Ve(rw) + 1e-12,
                        min(Ve(rhi), -1e-9) - 1e-12, xtol=1e-16, rtol=1e-15)
    a, b = tp(E)
    # period: weight (r-a)^-1/2 (b-r)^-1/2 times a smooth factor
    eps = 1e-7 * (b - a)

    def f(r):
        r = min(max(r, a + eps), b - eps)
        return math.sqrt((r - a) * (b - r) / (E - Ve(r)))
    val, _ = integrate.quad(f, a, b, weight="alg", wvar=(-0.5, -0.5), epsabs=0,
                            epsrel=1e-12, limit=400)
    return E, a, b, math.sqrt(2 * mu) * val


@pytest.mark.parametrize("v,j", [(0, 5), (2, 10), (4, 5), (10, 7)])
def test_rotating_levels_vs_scipy(orc, v, j):
    De, re, a = 0.1745, 1.40, 1.03
    s = orc.make_system(W.h2ca_system())
    mu, _, _ = orc.reduced_masses(s)
    V = lambda r: De * (1 - math.exp(-a * (r - re))) ** 2 - De
    E, rm, rp, tau = _scipy_level(V, mu, v, j, 0.3, 8.0)
    out = orc.level(s, v, j)
    assert out[0] == pytest.approx(E, rel=1e-11)
    assert out[1] == pytest.approx(rm, rel=1e-10)
    assert out[2] == pytest.approx(rp, rel=1e-10)
    assert out[3] == pytest.approx(tau, rel=1e-8)


def test_lj_level_count_vs_scipy(orc):
    """Generalized LJ molecule of the mixed surface: level v exists iff
    v + 1/2 is below the action at the dissociation limit (computed here with
    scipy quad)."""
    p = orc.make_pair(W.Pair("lj", {"n": 12, "m": 6, "eps": 0.02, "rm": 4.0}))
    m1, m2 = 7.0 * orc.AMU, 23.0 * orc.AMU
    mu = m1 * m2 / (m1 + m2)
    Cn, Cm = p.p[0], p.p[1]
    V = lambda r: Cn / r ** 12 - Cm / r ** 6
    rin = optimize.brentq(lambda r: V(r), 2.0, 4.0)
    val, _ = integrate.quad(lambda r: math.sqrt(max(-V(r), 0.0)), rin, 200.0, limit=800,
                            points=[4.0, 10.0, 30.0])
    I0 = math.sqrt(2 * mu) / math.pi * val
    vmax = int(math.floor(I0 - 0.5))
    assert 10 < vmax < 40
    rc, out = orc.level_pair(p, mu, vmax, 0)
    assert rc == 0 and out[0] < 0
    rc, _ = orc.level_pair(p, mu, vmax + 1, 0)
    assert rc == -2
    E, rm, rp, tau = _scipy_level(V, mu, 3, 4, 2.5, 40.0)
    rc, out = orc.level_pair(p, mu, 3, 4)
    assert rc == 0
    assert out[0] == pytest.approx(E, rel=1e-10)
    assert out[3] == pytest.approx(tau, rel=1e-8)


def test_buckingham_level_vs_scipy(orc):
    A, b, C6 = 50.0, 1.5, 40.0
    p = orc.make_pair(W.Pair("buck", {"A": A, "b": b, "C6": C6}))
    m1, m2 = 40.0 * orc.AMU, 7.0 * orc.AMU
    mu = m1 * m2 / (m1 + m2)
    V = lambda r: A * math.exp(-b * r) - C6 / r ** 6
    E, rm, rp, tau = _scipy_level(V, mu, 0, 2, 5.0, 40.0)
    rc, out = orc.level_pair(p, mu, 0, 2)
    assert rc == 0
    assert out[0] == pytest.approx(E, rel=1e-10)
    assert out[3] == pytest.approx(tau, rel=1e-8)
