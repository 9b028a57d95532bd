"""Colbert-Miller discrete variable representation (DVR) of the AB pair's
radial Hamiltonian, the paper's way of finding the molecule's internal
energy E(v, j) (Sec. 2.1; input keys npts, xmin, xmax of Sec. 3.1).

TEST INFRASTRUCTURE ONLY (part of the oracle): imported by tests, never by
the product path.

READING (the paper names the method and its grid keys only): the
particle-in-a-box form of Colbert and Miller (J. Chem. Phys. 96, 1982
(1992)) on (a, b) = (xmin, xmax) with N = npts + 1 intervals and the npts
interior points r_i = a + i (b - a) / N; kinetic matrix, with L = b - a,

    T_ii  = pi^2 / (4 mu L^2) [ (2 N^2 + 1) / 3 - 1 / sin^2(pi i / N) ]
    T_ii' = pi^2 / (4 mu L^2) (-1)^(i - i') [ 1 / sin^2(pi (i - i') / (2N))
                                              - 1 / sin^2(pi (i + i') / (2N)) ]

and the effective potential V(r_i) + j(j+1) / (2 mu r_i^2) on the diagonal.
E(v, j) is the (v+1)-th lowest eigenvalue (numpy's dense symmetric
eigensolver); it is a level of the pair if it lies below the top of the
centrifugal barrier (or below 0 without one).  The turning points and the
period at that energy come from the oracle's own routines, as for the
Bohr-Sommerfeld levels.
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as O


def kinetic(mu: float, a: float, b: float, npts: int):
    """(T, r): the kinetic matrix and the grid."""
    N = npts + 1
    L = b - a
    i = np.arange(1, N, dtype=np.float64)
    r = a + i * L / N
    I, J = np.meshgrid(i, i, indexing="ij")
    pref = math.pi ** 2 / (4.0 * mu * L * L)
    sign = np.where(((I - J) % 2) == 0, 1.0, -1.0)
    T = np.empty((npts, npts))
    off = ~np.eye(npts, dtype=bool)
    with np.errstate(divide="ignore"):     # the i = i' entries are replaced below
        full = pref * sign * (1.0 / np.sin(math.pi * (I - J) / (2 * N)) ** 2
                              - 1.0 / np.sin(math.pi * (I + J) / (2 * N)) ** 2)
    T[off] = full[off]
    d = np.arange(npts)
    T[d, d] = pref * ((2.0 * N * N + 1.0) / 3.0 - 1.0 / np.sin(math.pi * i / N) ** 2)
    return T, r


def hamiltonian(pair, mu: float, j: int, a: float, b: float, npts: int):
    T, r = kinetic(mu, a, b, npts)
    J2 = j * (j + 1.0)
    V = np.array([O.potential(pair, x)[0] for x in r]) + J2 / (2.0 * mu * r * r)
    return T + np.diag(V), r


def eigenvalues(pair, mu: float, j: int, a: float, b: float, npts: int):
    H, _ = hamiltonian(pair, mu, j, a, b, npts)
    return np.linalg.eigvalsh(H)


def level(sys, v: int, j: int, npts: int, a: float, b: float):
    """(E, r-, r+, tau) of level (v, j) of pair AB from the DVR energy."""
    mu12 = O.reduced_masses(sys)[0]
    pair = sys.pair[0]
    E = float(eigenvalues(pair, mu12, j, a, b, npts)[v])
    J2 = j * (j + 1.0)
    ok, rw, r0, hb = O.veff_extrema(pair, mu12, J2)
    if not ok:
        raise ValueError("no well for j = %d" % j)
    top = O.potential(pair, r0)[0] + J2 / (2.0 * mu12 * r0 * r0) if hb else 0.0
    if not E < top:
        raise ValueError("DVR level (v=%d, j=%d) is above the well" % (v, j))
    rc, rm, rp = O.turning_points(pair, mu12, J2, E, rw, r0)
    if rc != 0:
        raise ValueError("no turning points at the DVR energy")
    return np.array([E, rm, rp, O.period(pair, mu12, J2, E, rm, rp)])
