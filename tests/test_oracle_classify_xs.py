"""Pins of the oracle's product analysis (Sec. 2.2, Eq. (8)-(11)) and
aggregate step (Sec. 2.3 Eq. (12)-(16), Sec. 4 Eq. (18)-(19))."""
import math

import numpy as np
import pytest

import qcams_workloads as W


def _jacobi_from_cartesian(orc, sys, x, v):
    m = np.array([sys.mass[0], sys.mass[1], sys.mass[2]])
    mA, mB, mC = m
    mu12 = mA * mB / (mA + mB)
    mu123 = mC * (mA + mB) / m.sum()
    cm_x = (mA * x[0] + mB * x[1]) / (mA + mB)
    cm_v = (mA * v[0] + mB * v[1]) / (mA + mB)
    return np.concatenate([x[1] - x[0], x[2] - cm_x, mu12 * (v[1] - v[0]),
                           mu123 * (v[2] - cm_v)])


def _place(orc, sys, pair, r, far=50.0, vrel=0.0, vtan=0.0, vfar=1e-3):
    """Atoms of `pair` (0: AB, 1: BC, 2: CA) at distance r along x with relative
    radial speed vrel and tangential speed vtan; the third atom far away on z
    moving away."""
    idx = {0: (0, 1, 2), 1: (1, 2, 0), 2: (2, 0, 1)}[pair]
    i, k, third = idx
    x = np.zeros((3, 3))
    v = np.zeros((3, 3))
    x[k] = [r, 0.0, 0.0]
    v[k] = [vrel, vtan, 0.0]
    x[third] = [0.0, 0.0, far]
    v[third] = [0.0, 0.0, vfar]
    return _jacobi_from_cartesian(orc, sys, x, v)


def _pair_mu(sys, pair):
    m = [sys.mass[0], sys.mass[1], sys.mass[2]]
    a, b = [(0, 1), (1, 2), (2, 0)][pair]
    return m[a] * m[b] / (m[a] + m[b])


@pytest.mark.parametrize("pair,label", [(0, W.QUENCH), (2, W.R1), (1, W.R2)])
def test_channel_labels_and_vprime(orc, pair, label):
    """A single pair at the outer turning point of its level v, at rest:
    the label names that pair (r1 = AC + B, r2 = BC + A) and v' = v, j' = 0."""
    sw = W.System((1.008, 2.014, 40.078),
                  (W.Pair("morse", {"De": 0.1745, "re": 1.40, "alpha": 1.03}),
                   W.Pair("morse", {"De": 0.05, "re": 3.5, "alpha": 0.8}),
                   W.Pair("morse", {"De": 0.0625, "re": 3.78, "alpha": 0.62})))
    sys = orc.make_system(sw)
    prm = orc.make_params(W.Params())
    mu = _pair_mu(sys, pair)
    for v in (0, 1, 3):
        rc, lev = orc.level_pair(sys.pair[pair], mu, v, 0)
        assert rc == 0
        y = _place(orc, sys, pair, lev[2])
        c = orc.classify(sys, prm, y)
        assert c["label"] == label
        assert c["vt"] == v and c["jt"] == 0
        assert c["vprime"] == pytest.approx(v, abs=1e-9)
        assert c["jprime"] == pytest.approx(0.0, abs=1e-6)
        assert c["w"] == pytest.approx(1.0 / (prm.gb_sigma * math.sqrt(2 * math.pi)), rel=1e-6)


def test_rotating_pair_jprime_exact(orc):
    """Eq. (9): a pair with J^2 = j(j+1) gives j' = j."""
    sys = orc.make_system(W.h2ca_system())
    prm = orc.make_params(W.Params())
    mu = _pair_mu(sys, 2)
    for j in (1, 4, 9):
        rc, lev = orc.level_pair(sys.pair[2], mu, 1, j)
        assert rc == 0
        r = lev[2]
        vt = math.sqrt(j * (j + 1.0)) / (mu * r)
        y = _place(orc, sys, 2, r, vtan=vt)
        c = orc.classify(sys, prm, y)
        assert c["label"] == W.R1
        assert c["jt"] == j and abs(c["jprime"] - j) < 1e-9
        assert c["vt"] == 1 and c["vprime"] == pytest.approx(1.0, abs=1e-8)


def test_dissociation_and_unresolved(orc):
    sys = orc.make_system(W.h2ca_system())
    prm = orc.make_params(W.Params())
    # all three atoms far apart and flying apart
    x = np.array([[0.0, 0, 0], [40.0, 0, 0], [0, 0, 45.0]])
    v = np.array([[-1e-3, 0, 0], [1e-3, 0, 0], [0, 0, 1e-3]])
    c = orc.classify(sys, prm, _jacobi_from_cartesian(orc, sys, x, v))
    assert c["label"] == W.DISS
    assert (c["vt"], c["jt"], c["w"]) == (0, 0, 0.0)
    # AB pair just above its dissociation energy at short range: unbound
    mu = _pair_mu(sys, 0)
    Vr = 0.1745 * (1 - math.exp(-1.03 * (1.4 - 1.4))) ** 2 - 0.1745
    vrel = math.sqrt(2 * (1e-6 - Vr) / mu)
    c = orc.classify(sys, prm, _place(orc, sys, 0, 1.4, vrel=vrel))
    assert c["label"] == W.DISS
    vrel = math.sqrt(2 * (-1e-6 - Vr) / mu)
    c = orc.classify(sys, prm, _place(orc, sys, 0, 1.4, vrel=vrel))
    assert c["label"] == W.QUENCH
    # a compact triangle with all three pairs bound: unresolved
    x = np.array([[0.0, 0, 0], [1.4, 0, 0], [0.7, 3.7, 0]])
    c = orc.classify(sys, prm, _jacobi_from_cartesian(orc, sys, x, np.zeros((3, 3))))
    assert c["label"] == W.UNRESOLVED


def test_centrifugal_barrier_threshold(orc):
    """Eq. (8) with j' != 0: a rotating pair is bound below the top of its
    centrifugal barrier V_eff(r0) and unbound above it."""
    sys = orc.make_system(W.h2ca_system())
    prm = orc.make_params(W.Params())
    mu = _pair_mu(sys, 2)
    J2 = 40.0 * 41.0
    ok, rw, r0, hb = orc.veff_extrema(sys.pair[2], mu, J2)
    assert ok and hb and r0 > rw
    V0, dV0 = orc.potential(sys.pair[2], r0)
    assert dV0 == pytest.approx(J2 / (mu * r0 ** 3), rel=1e-9)   # V_eff'(r0) = 0
    top = V0 + J2 / (2 * mu * r0 * r0)
    assert top > 0.0
    r = rw
    Vr, _ = orc.potential(sys.pair[2], r)
    vtan = math.sqrt(J2) / (mu * r)
    for dE, expect in ((-1e-7, W.R1), (1e-7, W.DISS)):
        Ekin_rad = top + dE - Vr - J2 / (2 * mu * r * r)
        y = _place(orc, sys, 2, r, vrel=math.sqrt(2 * Ekin_rad / mu), vtan=vtan)
        c = orc.classify(sys, prm, y)
        assert c["label"] == expect
    # beyond the barrier, below its top: unbound (reading r < r0) unless literal
    r = r0 * 1.5
    Vr, _ = orc.potential(sys.pair[2], r)
    vtan = math.sqrt(J2) / (mu * r)
    Ekin_rad = top - 1e-5 - Vr - J2 / (2 * mu * r * r)
    y = _place(orc, sys, 2, r, vrel=math.sqrt(2 * Ekin_rad / mu), vtan=vtan, far=80.0)
    assert orc.classify(sys, prm, y)["label"] == W.DISS
    import dataclasses
    lit = orc.make_params(dataclasses.replace(W.Params(), literal_bound=1))
    assert orc.classify(sys, lit, y)["label"] == W.R1


def test_gb_weight(orc):
    """Eq. (11): normalised Gaussian about the nearest integer."""
    s = 0.04246609001440095
    w, vt = orc.gb_weight(3.0, s)
    assert vt == 3 and w == pytest.approx(1 / (s * math.sqrt(2 * math.pi)), rel=1e-15)
    w, vt = orc.gb_weight(2.49, s)
    assert vt == 2
    w, vt = orc.gb_weight(2.5, s)
    assert vt == 3
    # half maximum at +-0.05 (FWHM 0.1)
    w1, _ = orc.gb_weight(7.05, s)
    w0, _ = orc.gb_weight(7.0, s)
    assert w1 / w0 == pytest.approx(0.5, rel=1e-10)
    # integral over one bin is ~1
    xs = np.linspace(-0.5, 0.5, 20001)
    tot = np.trapezoid([orc.gb_weight(5 + x, s)[0] for x in xs], xs)
    assert tot == pytest.approx(1.0, rel=1e-6)


@pytest.mark.slow
def test_closed_channels_at_low_energy(orc):
    """Energetic thresholds: H2(v=0) + Ca at 1e4 K cannot react (needs
    ~32,000 K) or dissociate (~52,000 K), so every trajectory is quenched."""
    wl = W.config_small()
    sys = orc.make_system(wl.system)
    prm = orc.make_params(wl.params)
    I = wl.instances[0]
    lev = orc.level(sys, 0, 0)
    recs = orc.run_batch(sys, prm, orc.make_instance(I), lev, np.arange(40))
    assert set(recs["label"].tolist()) <= {W.QUENCH, W.UNRESOLVED}
    assert (recs["label"] == W.QUENCH).sum() >= 38
    # total energy E_0 + E_c = -0.1329 Eh lies between E_1 and E_2 of H2:
    # only v' <= 1 is open
    assert np.all(recs["vt"][recs["label"] == W.QUENCH] <= 1)


def test_large_impact_parameter_is_elastic(orc):
    """An atom passing far outside the interaction range leaves the molecule in
    its initial state."""
    sys = orc.make_system(W.h2ca_system())
    prm = orc.make_params(W.Params())
    inst = orc.make_instance(W.Instance(3.0e4, 2, 3, 10, 0, 11, W.B_FIXED, 28.0, 0.0))
    lev = orc.level(sys, 2, 3)
    recs = orc.run_batch(sys, prm, inst, lev, np.arange(3))
    assert np.all(recs["label"] == W.QUENCH)
    assert np.all(recs["vt"] == 2) and np.all(recs["jt"] == 3)
    assert np.allclose(recs["vprime"], 2.0, atol=1e-3)
    assert np.allclose(recs["jprime"], 3.0, atol=1e-3)


# --------------------------------------------------------------------------
# aggregate step
# --------------------------------------------------------------------------
def _toy_workload():
    inst = [W.Instance(1e4, 0, 0, 10, 0, 1, W.B_AREA, 0.0, 8.0),
            W.Instance(2e4, 0, 0, 10, 10, 1, W.B_AREA, 0.0, 5.0)]
    return W.Workload("toy", W.h2ca_system(), W.Params(), inst)


def test_opacity_and_error_eq16(orc):
    wl = _toy_workload()
    labels = np.array([0] * 10 + [0, 0, 0, 1, 1, 2, 3, 3, 3, 4])
    which = np.array([0] * 10 + [1] * 10)
    xs = orc.cross_sections(wl, labels, np.ones(20), which)
    assert np.all(xs["P"][0] == [1, 0, 0, 0]) and np.all(xs["dP"][0] == 0)
    assert xs["sigma"][0, 0] == pytest.approx(math.pi * 64.0, rel=1e-15)
    N = 10
    for c, Nx in enumerate([3, 2, 1, 3]):
        assert xs["P"][1, c] == pytest.approx(Nx / N, rel=1e-15)
        # Eq. (16)
        delta = math.sqrt(Nx) / N * math.sqrt((N - Nx) / N)
        assert xs["dP"][1, c] == pytest.approx(delta, rel=1e-12)
        assert xs["dsigma"][1, c] == pytest.approx(math.pi * 25.0 * delta, rel=1e-12)
    assert list(xs["counts"][1]) == [3, 2, 1, 3, 1, 0]
    # rate, Eq. (19): k = sigma sqrt(2 E_c / mu)
    sys = orc.make_system(wl.system)
    _, mu123, _ = orc.reduced_masses(sys)
    k = xs["sigma"][1, 0] * math.sqrt(2 * 2e4 * orc.KELVIN / mu123)
    assert xs["rate"][1, 0] == pytest.approx(k, rel=1e-14)


def test_weighted_estimator_reduces_to_plain(orc):
    wl = _toy_workload()
    rng = np.random.default_rng(0)
    labels = rng.integers(0, 4, 20)
    which = np.array([0] * 10 + [1] * 10)
    a = orc.cross_sections(wl, labels, np.ones(20), which)
    # constant weights scale P linearly
    b = orc.cross_sections(wl, labels, 2.0 * np.ones(20), which)
    assert np.allclose(b["P"], 2 * a["P"]) and np.allclose(b["dP"], 2 * a["dP"])


def test_sigma_from_grid_trapezoid(orc):
    """Eq. (18) (prefactor 2 pi): P = 1 on [0, bmax] gives the geometric
    cross section pi bmax^2 exactly with the trapezoid rule (linear integrand)."""
    b = np.arange(0, 5, 0.25)
    s, e = orc.sigma_from_grid(b, np.ones_like(b), np.zeros_like(b))
    assert s == pytest.approx(math.pi * b[-1] ** 2, rel=1e-14) and e == 0.0


def test_sigma_from_grid_error_closed_form(orc):
    """The error of Eq. (18) on a grid with nonzero per-b errors: on b = (0,
    1, 2) the trapezoid weights are (1/2, 1, 1/2), so with errors (d0, d1,
    d2) of P the error of sigma is 2 pi sqrt((1 d1)^2 + (1/2 * 2 d2)^2)
    (b = 0 contributes nothing); sigma itself is 2 pi (P1 + P2)."""
    b = np.array([0.0, 1.0, 2.0])
    P = np.array([0.9, 0.4, 0.1])
    d = np.array([0.03, 0.02, 0.05])
    s, e = orc.sigma_from_grid(b, P, d)
    assert s == pytest.approx(2 * math.pi * (0.4 + 0.1), rel=1e-15)
    assert e == pytest.approx(2 * math.pi * math.sqrt(0.02 ** 2 + 0.05 ** 2), rel=1e-15)
    # uneven spacing: b = (0.5, 1, 3): weights (1/4, 5/4, 1)
    b = np.array([0.5, 1.0, 3.0])
    s, e = orc.sigma_from_grid(b, P, d)
    w = np.array([0.25, 1.25, 1.0])
    assert s == pytest.approx(2 * math.pi * float((w * b * P).sum()), rel=1e-14)
    assert e == pytest.approx(2 * math.pi * math.sqrt(((w * b * d) ** 2).sum()), rel=1e-14)


def test_sigma_from_grid_error_is_the_spread_of_sigma(orc):
    """Independent errors propagate: with each P(b_k) drawn from a normal of
    width delta_k, the standard deviation of the trapezoid sigma over many
    draws is the stated error (within sampling error, 20,000 draws)."""
    rng = np.random.default_rng(11)
    b = np.arange(0, 5, 0.25)
    P = 0.6 * np.exp(-b / 2.0)
    d = rng.uniform(0.005, 0.04, b.size)
    s0, e0 = orc.sigma_from_grid(b, P, d)
    draws = np.array([orc.sigma_from_grid(b, P + d * rng.standard_normal(b.size), d)[0]
                      for _ in range(20000)])
    assert draws.mean() == pytest.approx(s0, abs=4 * e0 / math.sqrt(20000))
    # SD of a sample SD of n normals ~ sd / sqrt(2 n): 0.5 % here
    assert draws.std(ddof=1) == pytest.approx(e0, rel=0.02)


def test_gb_distribution_eq14_15(orc):
    wl = _toy_workload()
    labels = np.array([0, 0, 1, 3, 3] + [0] * 5 + [2] * 10)
    vt = np.array([0, 1, 2, 0, 0] + [0] * 5 + [3] * 10)
    w = np.array([9.0, 8.0, 7.0, 0.0, 0.0] + [1.0] * 5 + [2.0] * 10)
    which = np.array([0] * 10 + [1] * 10)
    H, Wt = orc.gb_distributions(wl, labels, vt, w, which)
    assert H[0, 0, 0] == 9.0 + 5.0 and H[0, 0, 1] == 8.0 and H[0, 1, 2] == 7.0
    assert Wt[0] == 9 + 8 + 7 + 5 + 2          # sum of weights plus N_d
    assert H[1, 2, 3] == 20.0 and Wt[1] == 20.0
