"""Pins of the oracle's random numbers (against numpy's independent
Philox4x64-10) and of the initial conditions of Sec. 2.1 (Eq. (5)-(7))."""
import math

import numpy as np
import pytest
from scipy import stats

import qcams_workloads as W

M64 = (1 << 64) - 1


def _numpy_philox(ctr, key):
    # numpy increments the 256-bit counter before each block
    c = (ctr[0] | (ctr[1] << 64) | (ctr[2] << 128) | (ctr[3] << 192)) - 1
    c %= 1 << 256
    g = np.random.Philox(counter=c, key=key[0] | (key[1] << 64))
    return [int(x) for x in g.random_raw(4)]


@pytest.mark.parametrize("ctr,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (230402733, 0)),
    ((123456789, 1, 0, 0), (230402732, 0)),
    ((M64, 0, 0, 0), (5, 0)),
    ((0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0, 0x082EFA98EC4E6C89),
     (0x452821E638D01377, 0xBE5466CF34E90C6C)),
])
def test_philox_matches_numpy(orc, ctr, key):
    assert orc.philox4x64_10(ctr, key) == _numpy_philox(ctr, key)


def test_uniform_stream(orc):
    seed = 230402731
    u = np.array([orc.uniforms(seed, i) for i in range(4000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    for c in range(6):
        assert stats.kstest(u[:, c], "uniform").pvalue > 1e-3
    # the six draws of one trajectory are the four words of block 0 and the
    # first two words of block 1
    raw0 = orc.philox4x64_10((7, 0, 0, 0), (seed, 0))
    raw1 = orc.philox4x64_10((7, 1, 0, 0), (seed, 0))
    u7 = orc.uniforms(seed, 7)
    expect = [(x >> 11) * 2.0 ** -53 for x in raw0] + [(x >> 11) * 2.0 ** -53 for x in raw1[:2]]
    assert list(u7) == expect


def _setup(orc, v=2, j=5, Ec=2.0e4, bmode=W.B_AREA, b=0.0, bmax=10.0):
    wl = W.config_batched()
    sys = orc.make_system(wl.system)
    prm = orc.make_params(wl.params)
    inst = orc.make_instance(W.Instance(Ec, v, j, 100, 0, 99, bmode, b, bmax))
    lev = orc.level(sys, v, j)
    return wl, sys, prm, inst, lev


@pytest.mark.parametrize("v,j", [(0, 0), (2, 5), (4, 0), (1, 9)])
def test_initial_state_invariants(orc, v, j):
    """Sec. 2.1: the molecule starts at its outer turning point with momentum
    perpendicular to rho1 and |P1| r+ = sqrt(j(j+1)) (Eq. (5)); its pair
    energy is E_vj; the atom starts at distance R of Eq. (6) with the
    collision momentum."""
    wl, sys, prm, inst, lev = _setup(orc, v, j)
    mu12, mu123, _ = orc.reduced_masses(sys)
    E, rm, rp, tau = lev
    Ec = inst.Ec_K * orc.KELVIN
    for tid in range(25):
        y, aux, smp = orc.init(sys, prm, inst, lev, tid)
        r1, r2, p1, p2 = y[0:3], y[3:6], y[6:9], y[9:12]
        assert np.linalg.norm(r1) == pytest.approx(rp, rel=1e-14)
        assert abs(r1 @ p1) <= 1e-13 * (1 + np.linalg.norm(p1))
        assert np.linalg.norm(p1) * rp == pytest.approx(math.sqrt(j * (j + 1.0)), rel=1e-13,
                                                        abs=1e-300)
        b, cth, phi, eta, chi, w = smp
        assert w == 1.0
        R = wl.params.R0 + chi * math.sqrt(2 * mu123 * Ec) * tau / mu123
        assert np.linalg.norm(r2) == pytest.approx(R, rel=1e-14)
        assert r2[1] == b and r2[0] == 0.0 and r2[2] < 0
        assert p2[0] == 0.0 and p2[1] == 0.0
        assert p2[2] == pytest.approx(math.sqrt(2 * mu123 * Ec), rel=1e-15)
        # pair energy of AB = E_vj (molecule alone)
        Eab = p1 @ p1 / (2 * mu12) + (0.1745 * (1 - math.exp(-1.03 * (rp - 1.4))) ** 2 - 0.1745)
        assert Eab == pytest.approx(E, rel=1e-12)
        # direction of rho1 from (theta, phi)
        assert r1[2] / rp == pytest.approx(cth, abs=1e-14)
        # aux: t, tmax = t_stop R / v_c, rstop shifted by R - R0
        vc = math.sqrt(2 * mu123 * Ec) / mu123
        assert aux[0] == 0.0
        assert aux[1] == pytest.approx(wl.params.t_stop * R / vc, rel=1e-14)
        assert aux[2] == pytest.approx(wl.params.r_stop + R - wl.params.R0, rel=1e-14)


def test_angle_and_impact_distributions(orc):
    """d(Omega) = sin(theta) dtheta dphi deta dchi (Sec. 2.3): cos(theta),
    phi, eta, chi uniform; area sampling makes b^2 uniform on [0, bmax^2]."""
    wl, sys, prm, inst, lev = _setup(orc, 0, 0)
    S = np.array([orc.init(sys, prm, inst, lev, t)[2] for t in range(3000)])
    b, cth, phi, eta, chi = S[:, 0], S[:, 1], S[:, 2], S[:, 3], S[:, 4]
    assert stats.kstest((b / 10.0) ** 2, "uniform").pvalue > 1e-3
    assert stats.kstest((cth + 1) / 2, "uniform").pvalue > 1e-3
    assert stats.kstest(phi / (2 * math.pi), "uniform").pvalue > 1e-3
    assert stats.kstest(eta / (2 * math.pi), "uniform").pvalue > 1e-3
    assert stats.kstest(chi, "uniform").pvalue > 1e-3
    # the direction of P1 relative to rho1 x z is uniform in eta: check the
    # rotational angular momentum direction is isotropic (mean ~ 0)
    wl, sys, prm, inst, lev = _setup(orc, 0, 4)
    L = []
    for t in range(2000):
        y, _, _ = orc.init(sys, prm, inst, lev, t)
        L.append(np.cross(y[0:3], y[6:9]))
    L = np.array(L) / math.sqrt(20.0)
    assert np.all(np.abs(L.mean(axis=0)) < 0.06)
    assert np.allclose(np.linalg.norm(L, axis=1), 1.0, rtol=1e-12)
    assert np.allclose((L ** 2).mean(axis=0), 1.0 / 3.0, atol=0.04)


def test_fixed_impact_parameter(orc):
    wl, sys, prm, inst, lev = _setup(orc, 0, 0, bmode=W.B_FIXED, b=2.25, bmax=0.0)
    for t in range(5):
        y, aux, smp = orc.init(sys, prm, inst, lev, t)
        assert smp[0] == 2.25 and y[4] == 2.25


def test_initial_state_classifies_as_its_level(orc):
    """The initial molecule, far from the atom, is quenched into its own
    level: j' = j exactly and v' = v to quadrature accuracy (Eq. (9)-(10))."""
    for v, j in [(0, 0), (2, 5), (4, 0), (3, 11)]:
        wl, sys, prm, inst, lev = _setup(orc, v, j)
        for t in range(3):
            y, aux, smp = orc.init(sys, prm, inst, lev, t)
            c = orc.classify(sys, prm, y)
            assert c["label"] == W.QUENCH
            assert c["jt"] == j and c["vt"] == v
            assert c["jprime"] == pytest.approx(j, abs=1e-12)
            assert c["vprime"] == pytest.approx(v, abs=1e-9)


def test_proposal_draws(orc):
    """Importance sampling over (b^2, chi, cos theta) cells: with a uniform
    table every weight is exactly 1 and the cells are uniform; with a skewed
    table the weights average to 1 (unbiasedness) and the cell frequencies
    follow the table."""
    K = 8192
    wl, sys, prm, inst, lev = _setup(orc, 0, 0)
    inst.b_mode = W.B_PROPOSAL
    q = np.ones(K)
    S = np.array([orc.init(sys, prm, inst, lev, t, prop_q=q)[2] for t in range(2000)])
    assert np.all(S[:, 5] == 1.0)
    assert stats.kstest((S[:, 0] / 10.0) ** 2, "uniform").pvalue > 1e-3
    assert stats.kstest((S[:, 1] + 1) / 2, "uniform").pvalue > 1e-3
    assert stats.kstest(S[:, 4], "uniform").pvalue > 1e-3
    rng = np.random.default_rng(3)
    q = rng.uniform(0.05, 1.0, K)
    q[:256] *= 20.0                     # favour the smallest impact parameters
    S = np.array([orc.init(sys, prm, inst, lev, t, prop_q=q)[2] for t in range(6000)])
    w = S[:, 5]
    assert abs(w.mean() - 1.0) < 4 * w.std() / np.sqrt(len(w))
    frac_small_b = ((S[:, 0] / 10.0) ** 2 < 1.0 / 32).mean()
    expect = q[:256].sum() / q.sum()
    assert abs(frac_small_b - expect) < 4 * np.sqrt(expect * (1 - expect) / len(w))
    # the weight is (1/K) / (q_k / sum q) of the drawn cell
    for t in range(20):
        smp = S[t]
        ib = min(int((smp[0] / 10.0) ** 2 * 32), 31)
        ichi = min(int(smp[4] * 16), 15)
        ic = min(int((smp[1] + 1) * 8), 15)
        k = (ib * 16 + ichi) * 16 + ic
        assert smp[5] == pytest.approx((1.0 / K) / (q[k] / q.sum()), rel=1e-12)
