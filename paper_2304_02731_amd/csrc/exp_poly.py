"""Coefficients of the polynomial that approximates e^r on [-ln2/2, ln2/2]
in the library's exp (qcams_device.h, exp_cw): interpolation of e^r at the
12 Chebyshev nodes of the interval (near-minimax), solved in 60-digit
arithmetic and printed as doubles, with the largest relative error of the
rounded coefficients (exact evaluation) over a dense grid.

    python paper_2304_02731_amd/csrc/exp_poly.py
"""
import mpmath as mp


def coefficients(deg: int = 11, digits: int = 60):
    mp.mp.dps = digits
    a = mp.log(2) / 2
    n = deg + 1
    nodes = [a * mp.cos(mp.pi * (2 * k + 1) / (2 * n)) for k in range(n)]
    A = mp.matrix([[x ** j for j in range(n)] for x in nodes])
    b = mp.matrix([mp.e ** x for x in nodes])
    c = mp.lu_solve(A, b)
    coef = [float(c[j]) for j in range(n)]
    worst = mp.mpf(0)
    for i in range(4001):
        r = -a + 2 * a * i / 4000
        p = mp.mpf(0)
        for cj in reversed(coef):
            p = p * r + mp.mpf(cj)
        worst = max(worst, abs(p / mp.e ** r - 1))
    return coef, float(worst)


if __name__ == "__main__":
    coef, worst = coefficients()
    for j, cj in enumerate(coef):
        print("c%-2d = %r" % (j, cj))
    print("largest relative error: %.3g" % worst)
