"""Pins of the oracle's Colbert-Miller DVR (the paper's internal-energy
method, Sec. 2.1): the kinetic matrix reproduces the particle-in-a-box
levels; on a box that holds the wavefunctions the Morse levels equal the
closed form of the Morse oscillator; rotating levels sit at the
Bohr-Sommerfeld ones to semiclassical accuracy; turning points at the DVR
energy."""
import math

import numpy as np
import pytest

import qcams_workloads as W


@pytest.fixture(scope="module")
def dvr(orc):
    from oracle import dvr as D
    return D


@pytest.mark.parametrize("mu,a,b,npts", [(918.7, 0.5, 10.0, 400), (1785.2, 1.0, 6.0, 250)])
def test_kinetic_matrix_is_the_box(dvr, mu, a, b, npts):
    """Alone, T is exact in the box's sine basis: its eigenvalues are
    k^2 pi^2 / (2 mu L^2), k = 1..npts."""
    T, r = dvr.kinetic(mu, a, b, npts)
    assert np.array_equal(T, T.T)
    assert r[0] > a and r[-1] < b and len(r) == npts
    ev = np.linalg.eigvalsh(T)
    k = np.arange(1, npts + 1)
    box = k ** 2 * math.pi ** 2 / (2.0 * mu * (b - a) ** 2)
    assert np.allclose(ev[:20], box[:20], rtol=1e-8, atol=0)
    assert np.allclose(ev, box, rtol=1e-6, atol=0)


def test_morse_levels_closed_form(orc, dvr):
    """H2 Morse on a box that holds the wavefunctions: E_v = -De + we (v+1/2)
    - we^2/(4 De) (v+1/2)^2 with we = alpha sqrt(2 De / mu)."""
    sys = orc.make_system(W.h2ca_system())
    mu = orc.reduced_masses(sys)[0]
    De, re, al = 0.1745, 1.40, 1.03
    ev = dvr.eigenvalues(sys.pair[0], mu, 0, 0.2, 10.0, 2000)
    we = al * math.sqrt(2.0 * De / mu)
    for v in range(8):
        ex = -De + we * (v + 0.5) - we * we / (4.0 * De) * (v + 0.5) ** 2
        assert ev[v] == pytest.approx(ex, rel=1e-11), v


def test_rotating_levels_near_bohr_sommerfeld(orc, dvr):
    """j > 0: DVR and Bohr-Sommerfeld levels agree to semiclassical accuracy,
    and the rotational energy grows with j."""
    sys = orc.make_system(W.h2ca_system())
    mu = orc.reduced_masses(sys)[0]
    prev = None
    for j in (0, 5, 10):
        ev = dvr.eigenvalues(sys.pair[0], mu, j, 0.2, 12.0, 1500)
        for v in range(4):
            bs = orc.level(sys, v, j)[0]
            # a factor-2 slip in the centrifugal term would move these by ~1e-2
            assert ev[v] == pytest.approx(bs, rel=1e-4), (v, j)
        if prev is not None:
            assert np.all(ev[:4] > prev[:4])
        prev = ev


def test_dvr_level_turning_points(orc, dvr):
    sys = orc.make_system(W.h2ca_system())
    mu = orc.reduced_masses(sys)[0]
    for v, j in [(0, 0), (3, 5), (6, 10)]:
        E, rm, rp, tau = dvr.level(sys, v, j, 1500, 0.2, 12.0)
        J2 = j * (j + 1.0)
        for r in (rm, rp):
            assert orc.potential(sys.pair[0], r)[0] + J2 / (2 * mu * r * r) == pytest.approx(E, abs=1e-12)
        bs = orc.level(sys, v, j)
        assert tau == pytest.approx(bs[3], rel=1e-3)     # period at a nearby energy
    with pytest.raises(ValueError):
        dvr.level(sys, 60, 0, 400, 0.2, 12.0)             # above the well
