// qcams_device.h -- device-side physics of the QCT hot path (HIP, gfx950).
//
// Koots & Perez-Rios, "PyQCAMS" (arXiv:2304.02731):
//   Sec. 2     Jacobi-coordinate Hamiltonian, Eq. (2); Hamilton's equations,
//              Eq. (3)-(4).
//   Sec. 2.1   initial conditions, Eq. (5)-(7).
//   Sec. 2.2   bound criterion Eq. (8); j' Eq. (9); v' Eq. (10); Gaussian
//              binning Eq. (11).
//   Sec. 3.2   Morse / generalized Lennard-Jones / Buckingham pairs; adaptive
//              Runge-Kutta 5(4) (Dormand-Prince).
//   Sec. 4     Morse form, Eq. (17).
//
// Everything here is FP64.  Functions are __host__ __device__ so that the same
// arithmetic can be exercised by host-side unit checks; the library itself
// only ever runs them inside kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dop853_tableau.h"

#define QD __host__ __device__ inline

namespace qd {

// ---------------------------------------------------------------------------
// constants
// ---------------------------------------------------------------------------
constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr int kNQ = 48;          // midpoint nodes of the radial quadrature
constexpr double kRFar = 1.0e5;  // outermost radius searched for a barrier (a0)

enum Kind { MORSE = 0, LJ = 1, BUCK = 2 };
// kernel specialisation code (never a pair's own kind): LJ with n = 12, m = 6
constexpr int LJ126 = 3;
enum Status { RUNNING = 0, OK_RSTOP = 1, OK_TMAX = 2, FAIL_MAXSTEPS = 3,
              FAIL_NONFINITE = 4, FAIL_HMIN = 5, COLLAPSE = 6 };
enum Label { QUENCH = 0, R1 = 1, R2 = 2, DISS = 3, UNRESOLVED = 4, FAILED = 5 };

// one pair interaction (Sec. 3.2)
struct Pot {
    int32_t kind, n, m, pad;
    double p0, p1, p2;   // MORSE {De, re, alpha} | LJ {Cn, Cm, -} | BUCK {A, b, C6}
};

// Shape of a pair potential beyond its inner limit, found once at set-up.
// With g(r) = r^3 V'(r), the effective potential V + J2/(2 mu r^2) has a
// stationary point where g(r) = J2/mu.  For the three families g is negative
// inside the potential minimum re and has a single maximum gmax at rstar
// beyond it, so J2/mu < gmax gives exactly one well (in (re, rstar)) and one
// centrifugal barrier (beyond rstar); J2/mu >= gmax gives no well.
struct Shape {
    double rin;     // Buckingham inner maximum (collapse radius), else 0
    double re;      // potential minimum
    double rstar;   // maximum of g beyond re
    double gmax;    // g(rstar)
};

struct Sys {
    Pot pot[3];       // AB, BC, CA
    Shape shape[3];
    double mu12, mu123, inv_mu12, inv_mu123;
    double mu_pair[3];
    double cA, cB;    // mA/(mA+mB), mB/(mA+mB)
    double rin2[3];   // squared collapse radii (0 when none)
};

struct Prm {
    double R0, t_stop, r_stop, atol, rtol, gb_sigma, h_fixed;
    int32_t fixed_step, literal_bound;
    int64_t max_steps;
    int32_t rk, pad;   // 0: Dormand-Prince 5(4); 1: Dormand-Prince 8(5,3)
};

// instance row as stored on the device (levels filled in at set-up)
struct Inst {
    double Ec;          // collision energy, hartree
    double b, bmax;
    int32_t b_mode, v, j, pad;
    int64_t n_traj, first_id;
    uint64_t seed;
    double Evj, rminus, rplus, tau;
    double Ec_K;        // collision energy as given, kelvin
};

// ---------------------------------------------------------------------------
// pair potentials with first and second derivatives
// ---------------------------------------------------------------------------
// finite test usable on host and device (x - x is NaN for inf and NaN)
QD bool is_finite(double x) { return x - x == 0.0; }

QD double ipow(double x, int n)
{
    double r = 1.0;
    while (n > 0) {
        if (n & 1) r *= x;
        x *= x;
        n >>= 1;
    }
    return r;
}

// ---------------------------------------------------------------------------
// fast FP64 helpers for the inner loop (hardware estimates refined by
// Newton or Goldschmidt steps)
// ---------------------------------------------------------------------------
// 1/x to about 2e-15 relative: the v_rcp_f64 estimate (5e-8) and one Newton step
// y <- y (2 - x y).  Used where that suffices: the error-norm weights (it
// moves the accept threshold err <= 1 by that much) and the centrifugal term
// of the radial quadrature.
QD double rcp_norm(double x)
{
    const double y = __builtin_amdgcn_rcp(x);
    return fma(y, fma(-x, y, 1.0), y);
}

// sqrt(s) and 1/(2 sqrt(s)) for s > 0: v_rsq_f64 estimate and two coupled
// Goldschmidt iterations (g -> sqrt(s), h -> 1/(2 sqrt(s))).
QD void sqrt_hrsqrt(double s, double& r, double& hr)
{
    const double y = __builtin_amdgcn_rsq(s);
    double g = s * y, h = 0.5 * y;
    double e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    r = g;
    hr = h;
}

// sqrt(s) and 1/sqrt(s) for s > 0
QD void sqrt_rsqrt(double s, double& r, double& ir)
{
    double h;
    sqrt_hrsqrt(s, r, h);
    ir = h + h;
}

// e^x for x < 709: Cody-Waite reduction x = n ln2 + r, |r| <= ln2/2, with
// ln2 split in a high part exact for |n| < 2^20 and a low correction, then a
// degree-11 polynomial in Horner form, scaled by 2^n.  n is the integer
// nearest to x log2(e), formed by one FMA against 1.5 * 2^52: the sum's ulp
// is 1, so the FMA rounds the exact product to an integer, and the low 32
// bits of the sum hold n in two's complement (|n| < 2^31), which the scaling
// takes directly.  The polynomial interpolates e^r at the 12 Chebyshev nodes
// of [-ln2/2, ln2/2] (solved in 60-digit arithmetic, csrc/exp_poly.py); with
// its coefficients rounded to double its relative error is below 1.7e-17,
// under the rounding of the evaluation itself.
QD double exp_cw(double x)
{
    const double kLog2e = 1.4426950408889634074;
    const double kLn2Hi = 6.93147180369123816490e-01;
    const double kLn2Lo = 1.90821492927058770002e-10;
    const double kShift = 6755399441055744.0;   // 1.5 * 2^52
    const double t = fma(x, kLog2e, kShift);
    const double n = t - kShift;
    double r = fma(-n, kLn2Hi, x);
    r = fma(-n, kLn2Lo, r);
    double p = 2.5110037605963777e-08;
    p = fma(p, r, 2.763263963904103e-07);
    p = fma(p, r, 2.755724091857897e-06);
    p = fma(p, r, 2.4801485482328494e-05);
    p = fma(p, r, 0.00019841269890047113);
    p = fma(p, r, 0.0013888888952314775);
    p = fma(p, r, 0.008333333333319601);
    p = fma(p, r, 0.0416666666664881);
    p = fma(p, r, 0.1666666666666668);
    p = fma(p, r, 0.5000000000000019);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)(unsigned)__builtin_bit_cast(unsigned long long, t));
}

// Step-size factor err^(-1/(q+1)) of the controller (q = 4 for the 5(4)
// pair, 7 for the 8(5,3) one), in FP32: a heuristic whose value only shapes
// the step sequence, never the accuracy bound.
template <int RK>
QD double ctrl_pow(double err)
{
    const float l = __builtin_amdgcn_logf((float)err);   // log2
    return (double)__builtin_amdgcn_exp2f((RK == 1 ? -0.125f : -0.2f) * l);
}

QD void pot_morse(const Pot& P, double r, double& V, double& d1, double& d2)
{
    const double De = P.p0, re = P.p1, a = P.p2;
    const double e = exp_cw(-a * (r - re));
    const double om = 1.0 - e;
    V = De * om * om - De;
    d1 = 2.0 * De * a * e * om;
    d2 = 2.0 * De * a * a * e * (2.0 * e - 1.0);
}

// Cn r^-n and Cm r^-m of the generalized LJ pair from ir = 1/r.  The 12-6
// form takes four multiplications; other exponents use binary powers, the
// power of m serving for n = 2m.
QD void lj_terms(const Pot& P, double ir, double& tn, double& tm)
{
    double pm, pn;
    if (P.n == 12 && P.m == 6) {
        const double i2 = ir * ir, i4 = i2 * i2;
        pm = i4 * i2;
        pn = pm * pm;
    } else {
        pm = ipow(ir, P.m);
        pn = P.n == 2 * P.m ? pm * pm : ipow(ir, P.n);
    }
    tn = P.p0 * pn;
    tm = P.p1 * pm;
}

QD void pot_lj(const Pot& P, double r, double& V, double& d1, double& d2)
{
    const double ir = 1.0 / r;
    double tn, tm;                            // Cn r^-n, Cm r^-m
    lj_terms(P, ir, tn, tm);
    V = tn - tm;
    d1 = (-P.n * tn + P.m * tm) * ir;
    d2 = ((P.n * (P.n + 1.0)) * tn - (P.m * (P.m + 1.0)) * tm) * ir * ir;
}

QD void pot_buck(const Pot& P, double r, double& V, double& d1, double& d2)
{
    const double A = P.p0, b = P.p1, C6 = P.p2;
    const double ir = 1.0 / r, ir2 = ir * ir, ir6 = ir2 * ir2 * ir2;
    const double ex = A * exp_cw(-b * r);
    V = ex - C6 * ir6;
    d1 = -b * ex + 6.0 * C6 * ir6 * ir;
    d2 = b * b * ex - 42.0 * C6 * ir6 * ir2;
}

QD void pot_all(const Pot& P, double r, double& V, double& d1, double& d2)
{
    if (P.kind == MORSE) pot_morse(P, r, V, d1, d2);
    else if (P.kind == LJ) pot_lj(P, r, V, d1, d2);
    else pot_buck(P, r, V, d1, d2);
}

QD double pot_V(const Pot& P, double r)
{
    double V, a, b;
    pot_all(P, r, V, a, b);
    return V;
}

// V'(r)/r for the force, specialised per kind at compile time (K >= 0) or
// selected at run time (K < 0; the kind is uniform across the wave).
// hr = 1/(2r): the Morse force takes it with a doubled constant (the same
// bits as 2 De alpha (e - e^2) / r), the other kinds double it.
template <int K>
QD double dV_over_r(const Pot& P, double r, double hr)
{
    const int kind = K >= 0 ? (K == LJ126 ? LJ : K) : P.kind;
    if (kind == MORSE) {
        // -alpha (r - re) as one FMA (alpha re is loop-invariant)
        const double e = exp_cw(fma(-P.p2, r, P.p2 * P.p1));
        return (4.0 * P.p0 * P.p2) * (e - e * e) * hr;
    }
    const double ir = hr + hr;
    if (kind == LJ) {
        double tn, tm;
        if (K == LJ126) {
            // the 12-6 branch of lj_terms, without the run-time test
            const double i2 = ir * ir, i4 = i2 * i2;
            const double pm = i4 * i2;
            tn = P.p0 * (pm * pm);
            tm = P.p1 * pm;
            return (-12.0 * tn + 6.0 * tm) * ir * ir;
        }
        lj_terms(P, ir, tn, tm);
        return (-P.n * tn + P.m * tm) * ir * ir;
    } else {
        const double ir2 = ir * ir, ir6 = ir2 * ir2 * ir2;
        return (-P.p1 * P.p0) * exp_cw(-P.p1 * r) * ir + (6.0 * P.p2) * ir6 * ir2;
    }
}

// ---------------------------------------------------------------------------
// Lane layouts of one trajectory.
//
// W = 1: one lane holds a whole trajectory; component arrays have six
//   entries, (rho1 x, y, z, rho2 x, y, z).
// W = 4: four consecutive lanes (a quad) share one trajectory.  Lane c < 3
//   holds spatial component c -- entries (rho1_c, rho2_c) -- and evaluates
//   pair c (AB, BC, CA) of the potential; lane 3 holds zeros and its pair
//   value is never read.  The squared distance of pair p is formed as
//   r_p+2^2 + (r_p+1^2 + r_p^2) over its components r (indices mod 3, FMAs)
//   in both layouts: in the quad, lane c also forms component c of pairs
//   c - 1 and c + 1, and lane p collects the other two components of its
//   own pair from lanes p + 1 and p + 2 with two rotations.  Error norms are summed as
//   (s_0 + s_1) + s_2 in both layouts (the quad adds s_3 = +0 to s_2, which
//   is exact for the non-negative terms summed here); every other operation
//   acts on one component with the same expression.  The layouts therefore
//   give bit-identical trajectories (with contraction limited to single
//   expressions, -ffp-contract=on).  W = 4 cuts the instructions a lane
//   issues per step to about 45 %, for the long trajectories whose latency
//   bounds a run.
// ---------------------------------------------------------------------------
template <int W> struct Lay;
// NC: spatial components per lane; N: state components (of x, and of p) per lane
template <> struct Lay<1> { static constexpr int NC = 3, N = 6; };
template <> struct Lay<4> { static constexpr int NC = 1, N = 2; };
template <> struct Lay<8> { static constexpr int NC = 1, N = 1; };

// RK coefficient tables live in constant memory (address space 4 on the
// device, read with scalar loads).
#if defined(__HIP_DEVICE_COMPILE__)
typedef __attribute__((address_space(4))) const double kcoef_t;
#else
typedef const double kcoef_t;
#endif

// A lane's part in its quad (W = 4 only).  Component c of pair q is
// fma(a_q, rho1_c, b_q rho2_c) with (a, b) = (1, 0), (-cA, 1), (-cB, -1) for
// AB, BC, CA (b rho2 is exact, so this rounds as the one-lane expressions).
struct Role {
    int c;          // spatial component and pair, 0..3
    int side;       // octet: 0 holds (rho1_c, P1_c), 1 holds (rho2_c, P2_c)
    Pot pot;        // pair c's potential (pair 0 for c = 3)
    double a[3];    // (a, b) of pairs c, c - 1, c + 1 (zeros on lane 3)
    double b[3];
    double rin2;    // pair c's squared collapse radius
    double im;      // octet: 1/mu of the lane's side
    double gam[3];  // octet: weights of g_AB r_AB, g_BC r_BC, g_CA r_CA in the side's force
    kcoef_t* kt;    // coefficient table of the step's RK variant
};

QD Role make_role(const Sys& S, int c, int side = 0)
{
    Role R;
    R.c = c;
    R.side = side;
    R.im = side ? S.inv_mu123 : S.inv_mu12;
    // -dV/drho1 = -g_AB r_AB + cA g_BC r_BC + cB g_CA r_CA; -dV/drho2 = -g_BC r_BC + g_CA r_CA
    R.gam[0] = side ? 0.0 : -1.0;
    R.gam[1] = side ? -1.0 : S.cA;
    R.gam[2] = side ? 1.0 : S.cB;
    for (int k = 0; k < 3; ++k) {
        const int q = c < 3 ? (k == 0 ? c : (k == 1 ? (c + 2) % 3 : (c + 1) % 3)) : -1;
        R.a[k] = q == 0 ? 1.0 : (q == 1 ? -S.cA : (q == 2 ? -S.cB : 0.0));
        R.b[k] = q == 1 ? 1.0 : (q == 2 ? -1.0 : 0.0);
    }
    R.rin2 = c == 1 ? S.rin2[1] : (c == 2 ? S.rin2[2] : S.rin2[0]);
    const Pot& a = S.pot[0];
    const Pot& b = S.pot[1];
    const Pot& e = S.pot[2];
    R.pot.kind = c == 1 ? b.kind : (c == 2 ? e.kind : a.kind);
    R.pot.n = c == 1 ? b.n : (c == 2 ? e.n : a.n);
    R.pot.m = c == 1 ? b.m : (c == 2 ? e.m : a.m);
    R.pot.pad = 0;
    R.pot.p0 = c == 1 ? b.p0 : (c == 2 ? e.p0 : a.p0);
    R.pot.p1 = c == 1 ? b.p1 : (c == 2 ? e.p1 : a.p1);
    R.pot.p2 = c == 1 ? b.p2 : (c == 2 ? e.p2 : a.p2);
    return R;
}

// Exchange inside a quad (DPP quad permutations; every lane of the quad
// active).  XOR1 swaps lanes (0,1),(2,3); XOR2 swaps (0,2),(1,3); BC<k>
// broadcasts lane k.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E;
template <int K> struct Bc { static constexpr int ctrl = K * 0x55; };
// lane l < 3 reads lane (l + 1) mod 3, resp. (l + 2) mod 3; lane 3 itself
constexpr int kDppNext = 0xC9, kDppPrev = 0xD2;

// (bound_ctrl set: no lane reads outside its quad, so no "old" value is
// needed and none is materialised)
template <int CTRL>
__device__ inline double quad_perm(double v)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ inline int quad_and(int v)
{
    v &= __builtin_amdgcn_mov_dpp(v, kDppXor1, 0xF, 0xF, true);
    return v & __builtin_amdgcn_mov_dpp(v, kDppXor2, 0xF, 0xF, true);
}

__device__ inline int quad_or(int v)
{
    v |= __builtin_amdgcn_mov_dpp(v, kDppXor1, 0xF, 0xF, true);
    return v | __builtin_amdgcn_mov_dpp(v, kDppXor2, 0xF, 0xF, true);
}

// Octets (eight lanes, two quads): DPP row shifts by four with bank masks.
// kOctLo: lanes of the first quad (banks 0, 2) read lane + 4; kOctHi: lanes
// of the second quad (banks 1, 3) read lane - 4; other lanes keep `old`.
constexpr int kDppShl4 = 0x104, kDppShr4 = 0x114, kBanksLo = 0x5, kBanksHi = 0xA;
template <int CTRL, int BANKS>
__device__ inline double oct_update(double old, double v)
{
    const unsigned long long o = __builtin_bit_cast(unsigned long long, old);
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp((int)(unsigned)o, (int)(unsigned)b, CTRL, 0xF, BANKS, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(unsigned)(o >> 32), (int)(unsigned)(b >> 32), CTRL,
                                               0xF, BANKS, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
// the value of the first quad's lane in both quads
__device__ inline double oct_from_lo(double v) { return oct_update<kDppShr4, kBanksHi>(v, v); }
// the value of the second quad's lane in both quads
__device__ inline double oct_from_hi(double v) { return oct_update<kDppShl4, kBanksLo>(v, v); }
// the partner's value (lane xor 4)
__device__ inline double oct_swap(double v)
{
    return oct_update<kDppShr4, kBanksHi>(oct_update<kDppShl4, kBanksLo>(v, v), v);
}
__device__ inline int oct_and(int v)
{
    const int s = __builtin_amdgcn_update_dpp(__builtin_amdgcn_update_dpp(v, v, kDppShl4, 0xF, kBanksLo, false),
                                              v, kDppShr4, 0xF, kBanksHi, false);
    return v & s;
}

// (s_0 + s_1) + (s_2 + s_3) over the quad, the same value in all four lanes
__device__ inline double quad_sum(double v)
{
    const double u = v + quad_perm<kDppXor1>(v);
    return u + quad_perm<kDppXor2>(u);
}

// ---------------------------------------------------------------------------
// Hamilton's equations (Eq. (3)-(4)) in separable form.
// x = (rho1, rho2), p = (P1, P2).  dx/dt = p / mu is linear, so only the
// force F(x) = -dV/dx is evaluated.  READING of the Jacobi signs (not fixed by
// the paper): rho1 = r_B - r_A, rho2 = r_C - R_cm(AB); pair vectors
// r_AB = rho1, r_BC = rho2 - cA rho1, r_CA = -rho2 - cB rho1.
// Outputs the squared pair distances (for the stop rules) as a by-product:
// all three in the one-lane layout, the lane's own pair in the quad.
// ---------------------------------------------------------------------------
template <int W, int K0, int K1, int K2>
QD void force_w(const Sys& S, const Role& R, const double* x, double* F, double* s2)
{
    constexpr int NC = Lay<W>::NC;
    // the octet gathers (rho1_c, rho2_c) in both of its quads, which then
    // work as the quad layout does
    double xs[2];
    const double* xx = x;
    if constexpr (W == 8) {
        xs[0] = oct_from_lo(x[0]);
        xs[1] = oct_from_hi(x[0]);
        xx = xs;
    }
    double rab[NC], rbc[NC], rca[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) {
        rab[a] = xx[a];
        rbc[a] = fma(-S.cA, xx[a], xx[NC + a]);
        rca[a] = fma(-S.cB, xx[a], -xx[NC + a]);
    }
    double sab = 0.0, sbc = 0.0, sca = 0.0, gab, gbc, gca;
    if constexpr (W == 1) {
        // pair p: r_p+2^2 + (r_p+1^2 + r_p^2) with component indices mod 3
        // (the quad's order)
        sab = fma(rab[2], rab[2], fma(rab[1], rab[1], rab[0] * rab[0]));
        sbc = fma(rbc[0], rbc[0], fma(rbc[2], rbc[2], rbc[1] * rbc[1]));
        sca = fma(rca[1], rca[1], fma(rca[0], rca[0], rca[2] * rca[2]));
        double dab, dbc, dca, hab, hbc, hca;   // distances, 1/(2 distance)
        sqrt_hrsqrt(sab, dab, hab);
        sqrt_hrsqrt(sbc, dbc, hbc);
        sqrt_hrsqrt(sca, dca, hca);
        gab = dV_over_r<K0>(S.pot[0], dab, hab);
        gbc = dV_over_r<K1>(S.pot[1], dbc, hbc);
        gca = dV_over_r<K2>(S.pot[2], dca, hca);
    } else {
        // component c of pairs c, c - 1, c + 1; pair p's other two
        // components gathered on lane p
        const double u0 = fma(R.a[0], xx[0], R.b[0] * xx[1]);
        const double u1 = fma(R.a[1], xx[0], R.b[1] * xx[1]);
        const double u2 = fma(R.a[2], xx[0], R.b[2] * xx[1]);
        const double v1 = quad_perm<kDppNext>(u1);   // component p + 1 of pair p
        const double v2 = quad_perm<kDppPrev>(u2);   // component p + 2 of pair p
        const double s = fma(v2, v2, fma(v1, v1, u0 * u0));
        sab = s;
        double d, hd;
        sqrt_hrsqrt(s, d, hd);
        // one kind for all pairs: one specialised path; a specialised triple
        // of kinds: each lane takes its pair's path (the wave runs all
        // three); otherwise the lane's own kind at run time
        double g;
        if constexpr (K0 >= 0 && K0 == K1 && K1 == K2) {
            g = dV_over_r<K0>(R.pot, d, hd);
        } else if constexpr (K0 >= 0 && K1 >= 0 && K2 >= 0) {
            if (R.c == 1) g = dV_over_r<K1>(R.pot, d, hd);
            else if (R.c == 2) g = dV_over_r<K2>(R.pot, d, hd);
            else g = dV_over_r<K0>(R.pot, d, hd);
        } else {
            g = dV_over_r<-1>(R.pot, d, hd);
        }
        gab = quad_perm<Bc<0>::ctrl>(g);
        gbc = quad_perm<Bc<1>::ctrl>(g);
        gca = quad_perm<Bc<2>::ctrl>(g);
    }
    if constexpr (W == 8) {
        // the side's force with per-lane weights: the same roundings as the
        // two expressions below (a zero weight adds an exact zero)
        F[0] = fma(R.gam[2] * gca, rca[0], fma(R.gam[1] * gbc, rbc[0], (R.gam[0] * gab) * rab[0]));
    } else {
        const double cgbc = S.cA * gbc, cgca = S.cB * gca;
#pragma unroll
        for (int a = 0; a < NC; ++a) {
            // -dV/drho1 = -g_AB r_AB + cA g_BC r_BC + cB g_CA r_CA
            F[a] = fma(cgca, rca[a], fma(cgbc, rbc[a], -gab * rab[a]));
            // -dV/drho2 = -g_BC r_BC + g_CA r_CA
            F[NC + a] = fma(gca, rca[a], -gbc * rbc[a]);
        }
    }
    s2[0] = sab;
    s2[1] = sbc;
    s2[2] = sca;
}

template <int K0, int K1, int K2>
QD void force(const Sys& S, const double* x, double* F, double* s2)
{
    force_w<1, K0, K1, K2>(S, Role{}, x, F, s2);
}

QD double hamiltonian(const Sys& S, const double* x, const double* p)
{
    double T = 0.0;
    for (int a = 0; a < 3; ++a) {
        T += 0.5 * p[a] * p[a] * S.inv_mu12;
        T += 0.5 * p[3 + a] * p[3 + a] * S.inv_mu123;
    }
    double r[3];
    double rbc[3], rca[3];
    for (int a = 0; a < 3; ++a) {
        rbc[a] = x[3 + a] - S.cA * x[a];
        rca[a] = -x[3 + a] - S.cB * x[a];
    }
    r[0] = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    r[1] = sqrt(rbc[0] * rbc[0] + rbc[1] * rbc[1] + rbc[2] * rbc[2]);
    r[2] = sqrt(rca[0] * rca[0] + rca[1] * rca[1] + rca[2] * rca[2]);
    return T + pot_V(S.pot[0], r[0]) + pot_V(S.pot[1], r[1]) + pot_V(S.pot[2], r[2]);
}

// ---------------------------------------------------------------------------
// Dormand-Prince 5(4), rewritten for the separable system.
//
// With v = p/mu and stage forces F_l, the stage positions are
//   X_i = x + h c_i v + (h^2/mu) sum_l (A^2)_il F_l
// and the step is
//   x' = x + h v + (h^2/mu) sum_l (bA)_l F_l,   p' = p + h sum_l b_l F_l,
// with error estimate
//   e_x = (h^2/mu) sum_l (eA)_l F_l,            e_p = h sum_l e_l F_l,
// e = b - bhat.  This is algebraically the same method as applying the
// tableau to the 12-component first-order system, but only the 6 force
// components of each stage are stored (half the registers).  X_7 = x', so
// F_7 is reused as F_1 of the next step (first same as last).
// ---------------------------------------------------------------------------
namespace dp {
// Butcher tableau of Dormand & Prince (1980)
constexpr double c2 = 1.0 / 5, c3 = 3.0 / 10, c4 = 4.0 / 5, c5 = 8.0 / 9;
constexpr double a21 = 1.0 / 5;
constexpr double a31 = 3.0 / 40, a32 = 9.0 / 40;
constexpr double a41 = 44.0 / 45, a42 = -56.0 / 15, a43 = 32.0 / 9;
constexpr double a51 = 19372.0 / 6561, a52 = -25360.0 / 2187, a53 = 64448.0 / 6561,
                 a54 = -212.0 / 729;
constexpr double a61 = 9017.0 / 3168, a62 = -355.0 / 33, a63 = 46732.0 / 5247,
                 a64 = 49.0 / 176, a65 = -5103.0 / 18656;
constexpr double b1 = 35.0 / 384, b3 = 500.0 / 1113, b4 = 125.0 / 192,
                 b5 = -2187.0 / 6784, b6 = 11.0 / 84;
constexpr double bh1 = 5179.0 / 57600, bh3 = 7571.0 / 16695, bh4 = 393.0 / 640,
                 bh5 = -92097.0 / 339200, bh6 = 187.0 / 2100, bh7 = 1.0 / 40;
constexpr double e1 = b1 - bh1, e3 = b3 - bh3, e4 = b4 - bh4, e5 = b5 - bh5,
                 e6 = b6 - bh6, e7 = -bh7;
// (A^2)_il = sum_j a_ij a_jl  (rows 3..6; row 2 is zero)
constexpr double q31 = a32 * a21;
constexpr double q41 = a42 * a21 + a43 * a31, q42 = a43 * a32;
constexpr double q51 = a52 * a21 + a53 * a31 + a54 * a41, q52 = a53 * a32 + a54 * a42,
                 q53 = a54 * a43;
constexpr double q61 = a62 * a21 + a63 * a31 + a64 * a41 + a65 * a51,
                 q62 = a63 * a32 + a64 * a42 + a65 * a52, q63 = a64 * a43 + a65 * a53,
                 q64 = a65 * a54;
// (bA)_l = sum_i b_i a_il
constexpr double w1 = b3 * a31 + b4 * a41 + b5 * a51 + b6 * a61;
constexpr double w2 = b3 * a32 + b4 * a42 + b5 * a52 + b6 * a62;
constexpr double w3 = b4 * a43 + b5 * a53 + b6 * a63;
constexpr double w4 = b5 * a54 + b6 * a64;
constexpr double w5 = b6 * a65;
// (eA)_l = sum_i e_i a_il  (row 7 of A is b)
constexpr double z1 = e3 * a31 + e4 * a41 + e5 * a51 + e6 * a61 + e7 * b1;
constexpr double z2 = e3 * a32 + e4 * a42 + e5 * a52 + e6 * a62;
constexpr double z3 = e4 * a43 + e5 * a53 + e6 * a63 + e7 * b3;
constexpr double z4 = e5 * a54 + e6 * a64 + e7 * b4;
constexpr double z5 = e6 * a65 + e7 * b5;
constexpr double z6 = e7 * b6;
}  // namespace dp

// ---------------------------------------------------------------------------
// RK coefficients in constant memory.  A step reads them through a pointer
// made opaque to the compiler once per step (an empty asm on it), so they
// are fetched inside the step loop with wide scalar loads (16 dwords per
// instruction) rather than held live across the loop, where they exceed the
// scalar registers and spill.  Each table lists the nonzero coefficients in
// the order the step uses them, so consecutive reads merge.
// ---------------------------------------------------------------------------

namespace dp {
enum : int {
    C2, C3, Q31, C4, Q41, Q42, C5, Q51, Q52, Q53, Q61, Q62, Q63, Q64,
    W1, W2, W3, W4, W5, B1, B3, B4, B5, B6, Z1, Z2, Z3, Z4, Z5, Z6,
    E1, E3, E4, E5, E6, E7, NV
};
struct Vals { double v[NV]; };
constexpr Vals vals()
{
    return Vals{{c2, c3, q31, c4, q41, q42, c5, q51, q52, q53, q61, q62, q63, q64,
                 w1, w2, w3, w4, w5, b1, b3, b4, b5, b6, z1, z2, z3, z4, z5, z6,
                 e1, e3, e4, e5, e6, e7}};
}
constexpr Vals VALS = vals();
}  // namespace dp
static __constant__ dp::Vals kDp = dp::vals();

// The table pointer, opaque to the compiler from here on: the coefficients
// are read afresh in every step instead of being hoisted out of the step loop.
QD kcoef_t* opaque_table(kcoef_t* k)
{
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+s"(k));
#endif
    return k;
}

// acc + a b, or a b alone for the first term of a sum (a product, not an
// FMA with a zero addend: the same value, counted as one operation)
QD double mac(bool first, double a, double b, double acc)
{
    return first ? a * b : fma(a, b, acc);
}

// Sum over the spatial components c of per-component partial sums, in the
// tree shared by both layouts (lane 3 of a quad contributes +0).
template <int W>
QD double comp_sum(const Role& R, const double* part)
{
    if constexpr (W == 1) {
        return (part[0] + part[1]) + part[2];
    } else if constexpr (W == 4) {
        return quad_sum(R.c < 3 ? part[0] : 0.0);
    } else {
        // the second quad holds the complete per-component sums
        return oct_from_hi(quad_sum(R.c < 3 ? part[0] : 0.0));
    }
}

// One trial step.  In: x, p, F1 = F(x), h.  Out: xn, pn, F7 = F(xn), the
// squared pair distances at xn, and the RMS error norm of Hairer-Norsett-
// Wanner (I, Sec. II.4) over the 12 components, scaled by
// atol + rtol max(|y|, |y'|).
template <int W, int K0, int K1, int K2>
QD double dopri5_trial(const Sys& S, const Role& R, const double* x, const double* p,
                       const double* F1, double h, double atol, double rtol, double* xn,
                       double* pn, double* F7, double* s2)
{
    using namespace dp;
    constexpr int NC = Lay<W>::NC, N = Lay<W>::N;
    kcoef_t* K = opaque_table(R.kt);
    double X[N], F2[N], F3[N], F4[N], F5[N], F6[N], junk[3];
    const double hh = h * h;
    // per-component 1/mu (uniform) and h^2/mu
    const double im0 = S.inv_mu12, im1 = S.inv_mu123;
    const double g0 = hh * im0, g1 = hh * im1;
    const double gR = hh * R.im;   // octet: the lane's side
#define IM(i) (W == 8 ? R.im : ((i) < NC ? im0 : im1))
#define GG(i) (W == 8 ? gR : ((i) < NC ? g0 : g1))
    // h v = h p / mu, formed once per step for the stage positions
    double hv[N];
#pragma unroll
    for (int i = 0; i < N; ++i) hv[i] = (h * IM(i)) * p[i];
#pragma unroll
    for (int i = 0; i < N; ++i) X[i] = fma(K[C2], hv[i], x[i]);
    force_w<W, K0, K1, K2>(S, R, X, F2, junk);
#pragma unroll
    for (int i = 0; i < N; ++i)
        X[i] = fma(GG(i), K[Q31] * F1[i], fma(K[C3], hv[i], x[i]));
    force_w<W, K0, K1, K2>(S, R, X, F3, junk);
#pragma unroll
    for (int i = 0; i < N; ++i)
        X[i] = fma(GG(i), fma(K[Q42], F2[i], K[Q41] * F1[i]), fma(K[C4], hv[i], x[i]));
    force_w<W, K0, K1, K2>(S, R, X, F4, junk);
#pragma unroll
    for (int i = 0; i < N; ++i)
        X[i] = fma(GG(i), fma(K[Q53], F3[i], fma(K[Q52], F2[i], K[Q51] * F1[i])),
                   fma(K[C5], hv[i], x[i]));
    force_w<W, K0, K1, K2>(S, R, X, F5, junk);
#pragma unroll
    for (int i = 0; i < N; ++i)
        X[i] = fma(GG(i), fma(K[Q64], F4[i], fma(K[Q63], F3[i], fma(K[Q62], F2[i], K[Q61] * F1[i]))),
                   fma(h * IM(i), p[i], x[i]));
    force_w<W, K0, K1, K2>(S, R, X, F6, junk);
    // step and error estimate (all but the F7 term) before the last force,
    // so that F2..F6 are dead when F7 is evaluated
    double ep[N], ex[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        xn[i] = fma(GG(i), fma(K[W5], F5[i], fma(K[W4], F4[i], fma(K[W3], F3[i], fma(K[W2], F2[i], K[W1] * F1[i])))),
                    fma(h * IM(i), p[i], x[i]));
        pn[i] = fma(h, fma(K[B6], F6[i], fma(K[B5], F5[i], fma(K[B4], F4[i], fma(K[B3], F3[i], K[B1] * F1[i])))),
                    p[i]);
        ex[i] = GG(i) * fma(K[Z6], F6[i], fma(K[Z5], F5[i], fma(K[Z4], F4[i],
                            fma(K[Z3], F3[i], fma(K[Z2], F2[i], K[Z1] * F1[i])))));
        ep[i] = fma(K[E6], F6[i], fma(K[E5], F5[i], fma(K[E4], F4[i], fma(K[E3], F3[i], K[E1] * F1[i]))));
    }
#undef IM
#undef GG
    force_w<W, K0, K1, K2>(S, R, xn, F7, s2);
    double part[NC];
    if constexpr (W == 8) {
        // the lane holds the k = side terms: the second quad continues the
        // first quad's partial sum of its component
        const double epi = fma(K[E7], F7[0], ep[0]);
        const double sx = fma(rtol, fmax(fabs(x[0]), fabs(xn[0])), atol);
        const double sp = fma(rtol, fmax(fabs(p[0]), fabs(pn[0])), atol);
        const double qx = ex[0] * rcp_norm(sx), qp = epi * (h * rcp_norm(sp));
        const double lo = oct_from_lo(fma(qx, qx, qp * qp));
        part[0] = fma(qx, qx, fma(qp, qp, lo));
    } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int i = c + k * NC;
                const double epi = fma(K[E7], F7[i], ep[i]);
                const double sx = fma(rtol, fmax(fabs(x[i]), fabs(xn[i])), atol);
                const double sp = fma(rtol, fmax(fabs(p[i]), fabs(pn[i])), atol);
                const double qx = ex[i] * rcp_norm(sx), qp = epi * (h * rcp_norm(sp));
                acc = fma(qx, qx, mac(k == 0, qp, qp, acc));
            }
            part[c] = acc;
        }
    }
    const double m = comp_sum<W>(R, part) * (1.0 / 12.0);
    double d, id;
    sqrt_rsqrt(m, d, id);
    return m > 0.0 ? d : m;   // 0, or NaN (rejected)
}

// ---------------------------------------------------------------------------
// Dormand-Prince 8(5,3), in the same separable form: with Q = A A,
//   X_i = x + h c_i v + (h^2/mu) sum_l Q_il F_l,
//   x'  = x + h v + (h^2/mu) sum_l (bA)_l F_l,     p' = p + h sum_l b_l F_l,
// and the two error estimates (5th and 3rd order, using F_13 = F(x'))
//   e_x = (h^2/mu) sum_l (E A + E_13 b)_l F_l,      e_p = h sum_l E_l F_l.
// The combined norm |e5|^2 / sqrt((|e5|^2 + 0.01 |e3|^2) n) is Hairer's.
// The derived coefficients are computed at compile time from the published
// tableau; zero products are dropped by the compiler.
// ---------------------------------------------------------------------------
namespace d8 {
constexpr int NS = 12;
struct Derived {
    double q[NS][NS];
    double bA[NS], e5A[NS], e3A[NS];
};
constexpr Derived derive()
{
    Derived d{};
    for (int i = 0; i < NS; ++i)
        for (int l = 0; l < NS; ++l) {
            double s = 0.0;
            for (int j = 0; j < NS; ++j) s += d8tab::A[i * NS + j] * d8tab::A[j * NS + l];
            d.q[i][l] = s;
        }
    for (int l = 0; l < NS; ++l) {
        double b = 0.0, e5 = 0.0, e3 = 0.0;
        for (int i = 0; i < NS; ++i) {
            b += d8tab::B[i] * d8tab::A[i * NS + l];
            e5 += d8tab::E5[i] * d8tab::A[i * NS + l];
            e3 += d8tab::E3[i] * d8tab::A[i * NS + l];
        }
        d.bA[l] = b;
        d.e5A[l] = e5 + d8tab::E5[NS] * d8tab::B[l];
        d.e3A[l] = e3 + d8tab::E3[NS] * d8tab::B[l];
    }
    return d;
}
constexpr Derived T = derive();
}  // namespace d8

namespace d8 {
// positions of the nonzero coefficients in the constant table (-1: zero)
constexpr int NV = 256;
struct Index {
    int16_t c[NS], q[NS][NS], bA[NS], b[NS], e5A[NS], e3A[NS], e5[NS], e3[NS];
    int16_t e5_13, e3_13, n;
};
struct Vals { double v[NV]; };
constexpr Index index()
{
    Index x{};
    int k = 0;
    for (int st = 0; st < NS; ++st) {
        x.c[st] = (int16_t)k++;
        for (int l = 0; l < NS; ++l)
            x.q[st][l] = (int16_t)((l < st && T.q[st][l] != 0.0) ? k++ : -1);
    }
    for (int l = 0; l < NS; ++l) {
        x.bA[l] = (int16_t)(T.bA[l] != 0.0 ? k++ : -1);
        x.b[l] = (int16_t)(d8tab::B[l] != 0.0 ? k++ : -1);
        x.e5A[l] = (int16_t)(T.e5A[l] != 0.0 ? k++ : -1);
        x.e3A[l] = (int16_t)(T.e3A[l] != 0.0 ? k++ : -1);
        x.e5[l] = (int16_t)(d8tab::E5[l] != 0.0 ? k++ : -1);
        x.e3[l] = (int16_t)(d8tab::E3[l] != 0.0 ? k++ : -1);
    }
    x.e5_13 = (int16_t)k++;
    x.e3_13 = (int16_t)k++;
    x.n = (int16_t)k;
    return x;
}
constexpr Index IX = index();
// first nonzero position of a coefficient row (the sum starts with a product)
constexpr int first_nz(const int16_t (&row)[NS])
{
    for (int l = 0; l < NS; ++l)
        if (row[l] >= 0) return l;
    return NS;
}
static_assert(IX.n <= NV, "coefficient table too small");
constexpr Vals vals()
{
    Vals v{};
    for (int st = 0; st < NS; ++st) {
        v.v[IX.c[st]] = d8tab::C[st];
        for (int l = 0; l < NS; ++l)
            if (IX.q[st][l] >= 0) v.v[IX.q[st][l]] = T.q[st][l];
    }
    for (int l = 0; l < NS; ++l) {
        if (IX.bA[l] >= 0) v.v[IX.bA[l]] = T.bA[l];
        if (IX.b[l] >= 0) v.v[IX.b[l]] = d8tab::B[l];
        if (IX.e5A[l] >= 0) v.v[IX.e5A[l]] = T.e5A[l];
        if (IX.e3A[l] >= 0) v.v[IX.e3A[l]] = T.e3A[l];
        if (IX.e5[l] >= 0) v.v[IX.e5[l]] = d8tab::E5[l];
        if (IX.e3[l] >= 0) v.v[IX.e3[l]] = d8tab::E3[l];
    }
    v.v[IX.e5_13] = d8tab::E5[NS];
    v.v[IX.e3_13] = d8tab::E3[NS];
    return v;
}
constexpr Vals VALS = vals();
}  // namespace d8
static __constant__ d8::Vals kD8 = d8::vals();

// The coefficient table of RK variant RK (1: DOP853, else DOPRI5).  Taken
// once per kernel and kept in scalar registers, so a step does not fetch the
// table's address again.
template <int RK>
QD kcoef_t* coef_table()
{
#if defined(__HIP_DEVICE_COMPILE__)
    return RK == 1 ? (kcoef_t*)&kD8.v[0] : (kcoef_t*)&kDp.v[0];
#else
    return RK == 1 ? &d8::VALS.v[0] : &dp::VALS.v[0];
#endif
}

template <int RK>
QD Role with_table(Role R)
{
    R.kt = coef_table<RK>();
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" : "+s"(R.kt));
#endif
    return R;
}

template <int W, int K0, int K1, int K2>
QD double dop853_trial(const Sys& S, const Role& R, const double* x, const double* p,
                       const double* F1, double h, double atol, double rtol, double* xn,
                       double* pn, double* F13, double* s2)
{
    using namespace d8;
    constexpr int NC = Lay<W>::NC, N = Lay<W>::N;
    kcoef_t* K = opaque_table(R.kt);
    double F[NS][N], junk[3];
    const double hh = h * h;
    const double im0 = S.inv_mu12, im1 = S.inv_mu123;
    const double g0 = hh * im0, g1 = hh * im1;
    const double gR = hh * R.im;   // octet: the lane's side
#define IM(i) (W == 8 ? R.im : ((i) < NC ? im0 : im1))
#define GG(i) (W == 8 ? gR : ((i) < NC ? g0 : g1))
#pragma unroll
    for (int i = 0; i < N; ++i) F[0][i] = F1[i];
    // h v = h p / mu, formed once per step for the stage positions
    double hv[N];
#pragma unroll
    for (int i = 0; i < N; ++i) hv[i] = (h * IM(i)) * p[i];
#pragma unroll
    for (int st = 1; st < NS; ++st) {
        double X[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double acc = 0.0;
            bool any = false;
#pragma unroll
            for (int l = 0; l < NS; ++l)
                if (IX.q[st][l] >= 0) {
                    acc = mac(!any, K[IX.q[st][l]], F[l][i], acc);
                    any = true;
                }
            X[i] = fma(K[IX.c[st]], hv[i], x[i]);
            if (any) X[i] = fma(GG(i), acc, X[i]);
        }
        force_w<W, K0, K1, K2>(S, R, X, F[st], junk);
    }
    // the step's six coefficient sums, each in l order (coefficient order)
    double sx[N], sp[N], a5[N], a3[N], b5[N], b3[N];
#pragma unroll
    for (int l = 0; l < NS; ++l) {
        const bool fx = IX.bA[l] >= 0 && l == first_nz(IX.bA), fp = IX.b[l] >= 0 && l == first_nz(IX.b);
        const bool f5 = IX.e5A[l] >= 0 && l == first_nz(IX.e5A), f3 = IX.e3A[l] >= 0 && l == first_nz(IX.e3A);
        const bool g5 = IX.e5[l] >= 0 && l == first_nz(IX.e5), g3 = IX.e3[l] >= 0 && l == first_nz(IX.e3);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            if (IX.bA[l] >= 0) sx[i] = mac(fx, K[IX.bA[l]], F[l][i], sx[i]);
            if (IX.b[l] >= 0) sp[i] = mac(fp, K[IX.b[l]], F[l][i], sp[i]);
            if (IX.e5A[l] >= 0) a5[i] = mac(f5, K[IX.e5A[l]], F[l][i], a5[i]);
            if (IX.e3A[l] >= 0) a3[i] = mac(f3, K[IX.e3A[l]], F[l][i], a3[i]);
            if (IX.e5[l] >= 0) b5[i] = mac(g5, K[IX.e5[l]], F[l][i], b5[i]);
            if (IX.e3[l] >= 0) b3[i] = mac(g3, K[IX.e3[l]], F[l][i], b3[i]);
        }
    }
    double ex5[N], ex3[N], ep5[N], ep3[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        xn[i] = fma(GG(i), sx[i], fma(h * IM(i), p[i], x[i]));
        pn[i] = fma(h, sp[i], p[i]);
        ex5[i] = GG(i) * a5[i];
        ex3[i] = GG(i) * a3[i];
        ep5[i] = b5[i];
        ep3[i] = b3[i];
    }
#undef IM
#undef GG
    force_w<W, K0, K1, K2>(S, R, xn, F13, s2);
    double part5[NC], part3[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double n5 = 0.0, n3 = 0.0;
#pragma unroll
        for (int k = 0; k < (W == 8 ? 1 : 2); ++k) {
            const int i = c + k * NC;
            // (the h of the momentum errors folded into their weight)
            const double e5p = fma(K[IX.e5_13], F13[i], ep5[i]);
            const double e3p = fma(K[IX.e3_13], F13[i], ep3[i]);
            const double isx = rcp_norm(fma(rtol, fmax(fabs(x[i]), fabs(xn[i])), atol));
            const double isp = h * rcp_norm(fma(rtol, fmax(fabs(p[i]), fabs(pn[i])), atol));
            const double a = ex5[i] * isx, b = e5p * isp, cc = ex3[i] * isx, d = e3p * isp;
            if constexpr (W == 8) {
                // the lane holds the k = side terms: the second quad continues
                // the first quad's partial sums of its component
                const double lo5 = oct_from_lo(fma(a, a, b * b));
                const double lo3 = oct_from_lo(fma(cc, cc, d * d));
                n5 = fma(a, a, fma(b, b, lo5));
                n3 = fma(cc, cc, fma(d, d, lo3));
            } else {
                n5 = fma(a, a, mac(k == 0, b, b, n5));
                n3 = fma(cc, cc, mac(k == 0, d, d, n3));
            }
        }
        part5[c] = n5;
        part3[c] = n3;
    }
    const double n5 = comp_sum<W>(R, part5), n3 = comp_sum<W>(R, part3);
    if (n5 == 0.0 && n3 == 0.0) return 0.0;
    double d, id;
    sqrt_rsqrt((n5 + 0.01 * n3) * 12.0, d, id);
    return n5 * id;
}

// Starting step (Hairer-Norsett-Wanner I, Sec. II.4), on the 12-component
// system y = (x, p), f = (p/mu, F).
template <int K0, int K1, int K2, int RK = 0>
QD double initial_step(const Sys& S, const double* x, const double* p, const double* F0,
                       double atol, double rtol, double span)
{
    const double im[6] = {S.inv_mu12, S.inv_mu12, S.inv_mu12,
                          S.inv_mu123, S.inv_mu123, S.inv_mu123};
    double d0 = 0.0, d1 = 0.0;
    for (int i = 0; i < 6; ++i) {
        const double sx = atol + rtol * fabs(x[i]), sp = atol + rtol * fabs(p[i]);
        const double vx = p[i] * im[i];
        d0 += (x[i] / sx) * (x[i] / sx) + (p[i] / sp) * (p[i] / sp);
        d1 += (vx / sx) * (vx / sx) + (F0[i] / sp) * (F0[i] / sp);
    }
    d0 = sqrt(d0 / 12.0);
    d1 = sqrt(d1 / 12.0);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    h0 = fmin(h0, span);
    double x1[6], p1[6], F1[6], s2[3];
    for (int i = 0; i < 6; ++i) {
        x1[i] = x[i] + h0 * p[i] * im[i];
        p1[i] = p[i] + h0 * F0[i];
    }
    force<K0, K1, K2>(S, x1, F1, s2);
    double d2 = 0.0;
    for (int i = 0; i < 6; ++i) {
        const double sx = atol + rtol * fabs(x[i]), sp = atol + rtol * fabs(p[i]);
        const double dvx = (p1[i] - p[i]) * im[i], dF = F1[i] - F0[i];
        d2 += (dvx / sx) * (dvx / sx) + (dF / sp) * (dF / sp);
    }
    d2 = sqrt(d2 / 12.0) / h0;
    const double dm = fmax(d1, d2);
    const double h1 = dm <= 1e-15 ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / dm, RK == 1 ? 0.125 : 0.2);
    return fmin(fmin(100.0 * h0, h1), span);
}

// ---------------------------------------------------------------------------
// Per-lane trajectory state kept in registers while in flight (the lane's
// components only in the quad layout; the scalars in every lane).
// ---------------------------------------------------------------------------
template <int W>
struct LaneW {
    double x[Lay<W>::N], p[Lay<W>::N], F[Lay<W>::N];
    double t, tmax, rstop2, h;
    int32_t nstep, nrej, status, last_rej;
};
using Lane = LaneW<1>;

// Advance one trajectory by one trial step of the adaptive RK integrator and
// apply the stop rules (READING of Sec. 3.1: stop after the first accepted
// step with the largest pair distance beyond r_stop_eff -- squares compared
// --, or at t_max; fail on step count, non-finite state, step-size
// underflow, or a pair inside a Buckingham inner maximum).  Step control:
// accept iff err <= 1, h <- h min(10, max(0.2, 0.9 err^-1/(q+1))), no
// increase right after a rejection, h_min = 1e-12 t_max.  In the quad
// layout all four lanes take the same decisions from the same values.
template <int W, int K0, int K1, int K2, int RK = 0>
QD void lane_step_w(const Sys& S, const Role& R, const Prm& P, LaneW<W>& L)
{
    constexpr int N = Lay<W>::N;
    double xn[N], pn[N], Fn[N], s2[3];
    const double span = L.tmax - L.t;
    const double hs = fmin(L.h, span);
    double err = RK == 1
        ? dop853_trial<W, K0, K1, K2>(S, R, L.x, L.p, L.F, hs, P.atol, P.rtol, xn, pn, Fn, s2)
        : dopri5_trial<W, K0, K1, K2>(S, R, L.x, L.p, L.F, hs, P.atol, P.rtol, xn, pn, Fn, s2);
    if (P.fixed_step) err = 0.0;
    if (!(err <= 1.0e300)) err = INFINITY;   // NaN or inf: reject
    const double pw = 0.9 * ctrl_pow<RK>(err);
    // Accept or reject by selects rather than branches: the tests below are
    // evaluated on every trial and take effect only on acceptance.
    const bool acc = err <= 1.0;
    // x - x is 0 for finite x, NaN otherwise
    double z = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const double zx = xn[i] - xn[i];
        const double zp = pn[i] - pn[i];
        z = z + zx;
        z = z + zp;
    }
    bool finite = z == 0.0;
    bool collapsed, far;
    if constexpr (W >= 4) {
        const int f = quad_and(finite ? 1 : 0);
        finite = (W == 8 ? oct_and(f) : f) != 0;
        // each lane tests its own pair; lane 3 has none
        const int own = R.c < 3 ? ((s2[0] < R.rin2 ? 1 : 0) | (s2[0] > L.rstop2 ? 2 : 0)) : 0;
        const int any = quad_or(own);
        collapsed = (any & 1) != 0;
        far = (any & 2) != 0;
    } else {
        collapsed = s2[0] < S.rin2[0] || s2[1] < S.rin2[1] || s2[2] < S.rin2[2];
        far = fmax(s2[0], fmax(s2[1], s2[2])) > L.rstop2;
    }
    const double tn = (hs == span) ? L.tmax : L.t + hs;
    int st = L.status;
    if (!finite) st = FAIL_NONFINITE;
    else if (collapsed) st = COLLAPSE;
    else if (far) st = OK_RSTOP;
    else if (tn >= L.tmax) st = OK_TMAX;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        L.x[i] = acc ? xn[i] : L.x[i];
        L.p[i] = acc ? pn[i] : L.p[i];
        L.F[i] = acc ? Fn[i] : L.F[i];
    }
    L.t = acc ? tn : L.t;
    L.status = acc ? st : L.status;
    L.nstep += acc ? 1 : 0;
    L.nrej += acc ? 0 : 1;
    // new step: min(10, max(0.2, 0.9 err^-1/(q+1))) after an acceptance (10
    // for err = 0; no increase right after a rejection), max(0.2, ...) after
    // a rejection; a fixed step never changes (it is always accepted)
    double fac = acc ? (err == 0.0 ? 10.0 : fmin(10.0, fmax(0.2, pw))) : fmax(0.2, pw);
    if (acc && L.last_rej && fac > 1.0) fac = 1.0;
    if (!P.fixed_step) L.h = hs * fac;
    L.last_rej = acc ? 0 : 1;
    if (L.status == RUNNING && !P.fixed_step && L.h < 1e-12 * L.tmax) L.status = FAIL_HMIN;
    if (L.status == RUNNING && L.nstep >= P.max_steps) L.status = FAIL_MAXSTEPS;
}

template <int K0, int K1, int K2, int RK = 0>
QD void lane_step(const Sys& S, const Prm& P, Lane& L)
{
    lane_step_w<1, K0, K1, K2, RK>(S, with_table<RK>(Role{}), P, L);
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// ---------------------------------------------------------------------------
QD void mul128(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo)
{
    const unsigned __int128 w = (unsigned __int128)a * b;
    hi = (uint64_t)(w >> 64);
    lo = (uint64_t)w;
}

QD void philox4x64(uint64_t c[4], uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t h0, l0, h1, l1;
        mul128(M0, c[0], h0, l0);
        mul128(M1, c[2], h1, l1);
        const uint64_t n0 = h1 ^ c[1] ^ k0, n2 = h0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = l1;
        c[2] = n2;
        c[3] = l0;
        k0 += W0;
        k1 += W1;
    }
}

QD double to_unit(uint64_t u) { return (double)(u >> 11) * 0x1.0p-53; }

// Six uniforms of trajectory `id`: words 0-3 of block 0 (b, cos theta, phi,
// eta) and words 0-1 of block 1 (chi, proposal cell) of the stream keyed by
// (seed, 0), counter (id, block, 0, 0).
QD void uniforms6(uint64_t seed, int64_t id, double* u)
{
    uint64_t c[4] = {(uint64_t)id, 0, 0, 0};
    philox4x64(c, seed, 0);
    u[0] = to_unit(c[0]);
    u[1] = to_unit(c[1]);
    u[2] = to_unit(c[2]);
    u[3] = to_unit(c[3]);
    uint64_t d[4] = {(uint64_t)id, 1, 0, 0};
    philox4x64(d, seed, 0);
    u[4] = to_unit(d[0]);
    u[5] = to_unit(d[1]);
}

// proposal cells: 32 (b^2) x 16 (chi) x 16 (cos theta)
constexpr int kCellsB = 32, kCellsChi = 16, kCellsCos = 16;
constexpr int kCells = kCellsB * kCellsChi * kCellsCos;

// first cell whose cumulative probability exceeds u
QD int find_cell(const double* cdf, double u)
{
    int lo = 0, hi = kCells - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cdf[mid] > u) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Initial conditions (Sec. 2.1).  Fills x, p; returns t_max, r_stop_eff and
// the sampled (b, cos theta, phi, eta, chi).  Returns false if b >= R.
// READING: uniform d(Omega) measure (cos theta in [-1,1), phi, eta in [0,2pi),
// chi in [0,1)); b fixed or bmax sqrt(U); atom along +z with b along +y;
// t_max = t_stop R / v_c; r_stop_eff = r_stop + (R - R0).
// ---------------------------------------------------------------------------
QD bool initial_state(const Sys& S, const Prm& P, const Inst& I, int64_t id, double* x,
                      double* p, double& tmax, double& rstop, double* smp, const double* prop_q,
                      const double* prop_cdf)
{
    double u[6];
    uniforms6(I.seed, id, u);
    double b = I.b_mode == 1 ? I.bmax * sqrt(u[0]) : I.b;
    double cth = 2.0 * u[1] - 1.0;
    const double phi = 2.0 * kPi * u[2];
    const double eta = 2.0 * kPi * u[3];
    double chi = u[4];
    double w = 1.0;
    if (I.b_mode == 2) {
        // importance sampling: cell k with probability q_k, uniform inside
        // it; weight = (uniform cell probability) / q_k
        const int k = find_cell(prop_cdf, u[5]);
        const int ib = k / (kCellsChi * kCellsCos);
        const int ichi = (k / kCellsCos) % kCellsChi;
        const int ic = k % kCellsCos;
        b = I.bmax * sqrt((ib + u[0]) * (1.0 / kCellsB));
        cth = -1.0 + (ic + u[1]) * (2.0 / kCellsCos);
        chi = (ichi + u[4]) * (1.0 / kCellsChi);
        w = (1.0 / kCells) / prop_q[k];
    }
    const double sth = sqrt(1.0 - cth * cth);
    double sph, cph, set, cet;
    sincos(phi, &sph, &cph);
    sincos(eta, &set, &cet);
    const double rp = I.rplus;
    const double jj = (double)I.j;
    const double P1 = sqrt(jj * (jj + 1.0)) / rp;
    // Eq. (5): molecule at r+, momentum perpendicular to rho1
    x[0] = rp * sth * cph;
    x[1] = rp * sth * sph;
    x[2] = rp * cth;
    p[0] = P1 * (sph * cet - cth * cph * set);
    p[1] = P1 * (-cph * cet - cth * sph * set);
    p[2] = P1 * (sth * set);
    // Eq. (6): vibrational phase through the initial distance
    const double P2 = sqrt(2.0 * S.mu123 * I.Ec);
    const double R = P.R0 + chi * P2 * I.tau * S.inv_mu123;
    x[3] = 0.0;
    x[4] = b;
    x[5] = -sqrt(R * R - b * b);
    p[3] = 0.0;
    p[4] = 0.0;
    p[5] = P2;
    const double vc = P2 * S.inv_mu123;
    tmax = P.t_stop * R / vc;
    rstop = P.r_stop + (R - P.R0);
    smp[0] = b;
    smp[1] = cth;
    smp[2] = phi;
    smp[3] = eta;
    smp[4] = chi;
    smp[5] = w;
    return b < R;
}

// ---------------------------------------------------------------------------
// Radial structure of one pair: well, barrier, turning points, action, period
// ---------------------------------------------------------------------------
// g(r) = r^3 V'(r) and its derivative
QD void gfun(const Pot& P, double r, double& g, double& dg)
{
    double V, d1, d2;
    pot_all(P, r, V, d1, d2);
    g = r * r * r * d1;
    dg = r * r * (3.0 * d1 + r * d2);
}

// Root of g(r) = q on a bracket [lo, hi] where g - q changes sign, by Newton
// steps kept inside the bracket (bisection when Newton leaves it).
QD double solve_g(const Pot& P, double q, double lo, double hi)
{
    double glo, dg;
    gfun(P, lo, glo, dg);
    const bool inc = glo < q;   // g - q goes from - to + on [lo, hi]
    double r = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        double g;
        gfun(P, r, g, dg);
        const double f = g - q;
        if (f == 0.0) return r;
        if ((f < 0.0) == inc) lo = r; else hi = r;
        double rn = r - f / dg;
        if (!(rn > lo && rn < hi)) rn = 0.5 * (lo + hi);
        if (fabs(rn - r) <= 1e-15 * r || hi - lo <= 2e-16 * r) return rn;
        r = rn;
    }
    return r;
}

struct Radial {
    bool well;      // the effective potential has a well
    bool barrier;   // ... and an outer maximum within kRFar
    double rw, r0;  // well minimum, barrier (inf when none)
};

// Eq. (8)'s r0, "the local maximum of the effective potential", and the well.
QD Radial radial(const Pot& P, const Shape& Sh, double mu, double J2)
{
    Radial R;
    const double q = J2 / mu;
    R.well = false;
    R.barrier = false;
    R.rw = Sh.re;
    R.r0 = INFINITY;
    if (!(q < Sh.gmax)) return R;
    R.well = true;
    if (q <= 0.0) return R;
    R.rw = solve_g(P, q, Sh.re, Sh.rstar);
    double gfar, dg;
    gfun(P, kRFar, gfar, dg);
    if (gfar >= q) return R;    // no maximum inside kRFar: J2 -> 0 limit
    // bracket [rstar, hi] with g(hi) < q by doubling
    double lo = Sh.rstar, hi = 2.0 * Sh.rstar;
    for (int it = 0; it < 64; ++it) {
        double g;
        gfun(P, hi, g, dg);
        if (g < q || hi >= kRFar) break;
        lo = hi;
        hi = fmin(2.0 * hi, kRFar);
    }
    R.r0 = solve_g(P, q, lo, hi);
    R.barrier = true;
    return R;
}

QD double veff(const Pot& P, double mu, double J2, double r)
{
    return pot_V(P, r) + J2 / (2.0 * mu * r * r);
}

// Root of V_eff(r) = E on [lo, hi] (V_eff - E changes sign), Newton in a
// bracket.
QD double solve_veff(const Pot& P, double mu, double J2, double E, double lo, double hi)
{
    const bool inc = veff(P, mu, J2, lo) < E;
    double r = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        double V, d1, d2;
        pot_all(P, r, V, d1, d2);
        const double f = V + J2 / (2.0 * mu * r * r) - E;
        const double df = d1 - J2 / (mu * r * r * r);
        if (f == 0.0) return r;
        if ((f < 0.0) == inc) lo = r; else hi = r;
        double rn = r - f / df;
        if (!(rn > lo && rn < hi)) rn = 0.5 * (lo + hi);
        if (fabs(rn - r) <= 1e-15 * r || hi - lo <= 2e-16 * r) return rn;
        r = rn;
    }
    return r;
}

// Turning points r- < rw < r+ at energy E (E below the barrier top and above
// the well bottom).  Returns false when they cannot be bracketed.
QD bool turning_points(const Pot& P, const Shape& Sh, const Radial& R, double mu, double J2,
                       double E, double& rm, double& rp)
{
    if (!(veff(P, mu, J2, R.rw) < E)) return false;
    // inner bracket: shrink towards the inner limit until V_eff > E
    double lo = R.rw;
    bool ok = false;
    for (int it = 0; it < 80; ++it) {
        lo = Sh.rin > 0.0 ? Sh.rin + 0.5 * (lo - Sh.rin) : 0.5 * lo;
        if (veff(P, mu, J2, lo) > E) { ok = true; break; }
    }
    if (!ok) return false;
    double hi = R.rw;
    ok = false;
    const double top = R.barrier ? R.r0 : kRFar;
    for (int it = 0; it < 80; ++it) {
        hi = fmin(2.0 * hi, top);
        if (veff(P, mu, J2, hi) > E) { ok = true; break; }
        if (hi >= top) break;
    }
    if (!ok) return false;
    rm = solve_veff(P, mu, J2, E, lo, R.rw);
    rp = solve_veff(P, mu, J2, E, R.rw, hi);
    return true;
}

// Action and period between the turning points: with r = c + h cos(theta)
// the integrands of Eq. (10) and Eq. (7) become smooth, even and periodic in
// theta, so the midpoint rule converges geometrically.
//   act = (sqrt(2mu)/pi) int sqrt(E - V_eff) dr ; per = sqrt(2mu) int dr / sqrt(E - V_eff)
// ap_node gives one node's terms of the two sums (sin(theta) sqrt(E - V_eff)
// and sin(theta) / sqrt(E - V_eff)); ap_finish scales the sums.
QD void ap_node(const Pot& P, double cent, double E, double c, double h, double st, double ct,
                double& a, double& q)
{
    const double r = c + h * ct;
    const double ir = rcp_norm(r);
    const double kin = E - (pot_V(P, r) + cent * (ir * ir));
    a = 0.0;
    q = 0.0;
    if (kin > 0.0) {
        double sq, isq;
        sqrt_rsqrt(kin, sq, isq);
        a = st * sq;
        q = st * isq;
    }
}

QD void ap_finish(double mu, double h, double sa, double sp, double& act, double& per)
{
    const double s2mu = sqrt(2.0 * mu);
    act = s2mu / kPi * h * (kPi / kNQ) * sa;
    per = s2mu * h * (kPi / kNQ) * sp;
}

QD void action_period(const Pot& P, double mu, double J2, double E, double rm, double rp,
                      double& act, double& per)
{
    const double c = 0.5 * (rp + rm), h = 0.5 * (rp - rm);
    const double cent = J2 / (2.0 * mu);
    double sa = 0.0, sp = 0.0;
    // nodes theta_k = pi (k + 1/2) / kNQ by rotation from theta_0 (the
    // recurrence's rounding, a few ulp over kNQ steps, is far below the
    // error of the rule)
    double st, ct, sd, cd;
    sincos(kPi * 0.5 / kNQ, &st, &ct);
    sincos(kPi / kNQ, &sd, &cd);
    for (int k = 0; k < kNQ; ++k) {
        double a, q;
        ap_node(P, cent, E, c, h, st, ct, a, q);
        sa += a;
        sp += q;
        const double cn = fma(ct, cd, -st * sd);
        st = fma(st, cd, ct * sd);
        ct = cn;
    }
    ap_finish(mu, h, sa, sp, act, per);
}

// Bohr-Sommerfeld level of the AB molecule: E with act(E) = v + 1/2,
// safeguarded Newton using d act/dE = per/(2 pi).  Returns 0, or -2 when the
// level is not bound, -3 when a root cannot be bracketed.  `ap(J2, E, rm, rp,
// act, per)` evaluates the action and period (serially, or one node per lane
// of a wave).
template <class AP>
QD int bs_level_with(const Pot& P, const Shape& Sh, double mu, int v, int j, double* out,
                     const AP& ap)
{
    const double J2 = (double)j * (j + 1.0);
    const Radial R = radial(P, Sh, mu, J2);
    if (!R.well) return -2;
    const double Elo = veff(P, mu, J2, R.rw);
    const double Ehi = R.barrier ? veff(P, mu, J2, R.r0) : 0.0;
    const double target = v + 0.5;
    double lo = Elo, hi = Ehi - 1e-13 * fabs(Ehi - Elo);
    double rm, rp, act, per;
    if (!turning_points(P, Sh, R, mu, J2, hi, rm, rp)) return -2;
    ap(J2, hi, rm, rp, act, per);
    if (!(act > target)) return -2;
    // start from the harmonic estimate near the bottom of the well
    double E = lo + (hi - lo) * fmin(0.5, target / act);
    for (int it = 0; it < 200; ++it) {
        if (!turning_points(P, Sh, R, mu, J2, E, rm, rp)) return -3;
        ap(J2, E, rm, rp, act, per);
        const double f = act - target;
        if (f < 0.0) lo = E; else hi = E;
        double En = E - f * 2.0 * kPi / per;
        if (!(En > lo && En < hi)) En = 0.5 * (lo + hi);
        const bool done = fabs(En - E) <= 4e-16 * fabs(E) || hi - lo <= 4e-16 * fabs(E);
        E = En;
        if (done) break;
    }
    if (!turning_points(P, Sh, R, mu, J2, E, rm, rp)) return -3;
    ap(J2, E, rm, rp, act, per);
    out[0] = E;
    out[1] = rm;
    out[2] = rp;
    out[3] = per;
    return 0;
}

QD int bs_level(const Pot& P, const Shape& Sh, double mu, int v, int j, double* out)
{
    return bs_level_with(P, Sh, mu, v, j, out,
                         [&](double J2, double E, double rm, double rp, double& act, double& per) {
                             action_period(P, mu, J2, E, rm, rp, act, per);
                         });
}

// Turning points and period of the AB pair at a given energy E of level
// (v, j) (E from the DVR): out = E, r-, r+, tau.  Returns -2 when E is not
// inside the well of V_eff.
QD int level_at_energy(const Pot& P, const Shape& Sh, double mu, int j, double E, double* out)
{
    const double J2 = (double)j * (j + 1.0);
    const Radial R = radial(P, Sh, mu, J2);
    if (!R.well) return -2;
    const double Elo = veff(P, mu, J2, R.rw);
    const double Ehi = R.barrier ? veff(P, mu, J2, R.r0) : 0.0;
    if (!(E > Elo && E < Ehi)) return -2;
    double rm, rp, act, per;
    if (!turning_points(P, Sh, R, mu, J2, E, rm, rp)) return -3;
    action_period(P, mu, J2, E, rm, rp, act, per);
    out[0] = E;
    out[1] = rm;
    out[2] = rp;
    out[3] = per;
    return 0;
}

// ---------------------------------------------------------------------------
// Product analysis of one final state (Sec. 2.2)
// ---------------------------------------------------------------------------
struct Outcome {
    int label, vt, jt;
    double vprime, jprime, w;
};

QD Outcome classify_state(const Sys& S, const Prm& P, const double* x, const double* p)
{
    Outcome o;
    o.label = DISS;
    o.vt = 0;
    o.jt = 0;
    o.vprime = 0.0;
    o.jprime = 0.0;
    o.w = 0.0;
    double r[3][3], u[3][3];
    for (int a = 0; a < 3; ++a) {
        const double v1 = p[a] * S.inv_mu12, v2 = p[3 + a] * S.inv_mu123;
        r[0][a] = x[a];
        r[1][a] = x[3 + a] - S.cA * x[a];
        r[2][a] = -x[3 + a] - S.cB * x[a];
        u[0][a] = v1;
        u[1][a] = v2 - S.cA * v1;
        u[2][a] = -v2 - S.cB * v1;
    }
    double E[3], J2[3], d[3];
    Radial R[3];
    int nb = 0, which = -1;
    for (int k = 0; k < 3; ++k) {
        const double mu = S.mu_pair[k];
        d[k] = sqrt(r[k][0] * r[k][0] + r[k][1] * r[k][1] + r[k][2] * r[k][2]);
        const double v2 = u[k][0] * u[k][0] + u[k][1] * u[k][1] + u[k][2] * u[k][2];
        E[k] = 0.5 * mu * v2 + pot_V(S.pot[k], d[k]);
        const double Lx = r[k][1] * u[k][2] - r[k][2] * u[k][1];
        const double Ly = r[k][2] * u[k][0] - r[k][0] * u[k][2];
        const double Lz = r[k][0] * u[k][1] - r[k][1] * u[k][0];
        J2[k] = mu * mu * (Lx * Lx + Ly * Ly + Lz * Lz);
        R[k] = radial(S.pot[k], S.shape[k], mu, J2[k]);
        bool bound = false;
        if (R[k].well) {
            // Eq. (8): below the barrier top (0 when there is no maximum);
            // READING: unless literal, the pair must also be inside r0
            const double thr = (R[k].barrier && J2[k] > 0.0) ? veff(S.pot[k], mu, J2[k], R[k].r0)
                                                             : 0.0;
            bound = E[k] < thr && (P.literal_bound || d[k] < R[k].r0);
        }
        if (bound) {
            ++nb;
            which = k;
        }
    }
    if (nb == 0) return o;
    if (nb > 1) {
        o.label = UNRESOLVED;
        return o;
    }
    const int k = which;
    o.label = k == 0 ? QUENCH : (k == 2 ? R1 : R2);
    const double mu = S.mu_pair[k];
    // Eq. (9)
    o.jprime = -0.5 + 0.5 * sqrt(1.0 + 4.0 * J2[k]);
    o.jt = (int)floor(o.jprime + 0.5);
    // Eq. (10) with E'_int = the pair energy
    double rm, rp, act, per;
    if (!turning_points(S.pot[k], S.shape[k], R[k], mu, J2[k], E[k], rm, rp)) {
        o.label = UNRESOLVED;
        o.jt = 0;
        o.jprime = 0.0;
        return o;
    }
    action_period(S.pot[k], mu, J2[k], E[k], rm, rp, act, per);
    o.vprime = act - 0.5;
    // Eq. (11): Gaussian weight about the nearest integer
    const double n = floor(o.vprime + 0.5);
    o.vt = (int)n;
    const double dv = o.vprime - n, sg = P.gb_sigma;
    o.w = exp(-dv * dv / (2.0 * sg * sg)) / (sg * sqrt(2.0 * kPi));
    return o;
}

// ---------------------------------------------------------------------------
// Set-up of the pair shapes (inner limit, minimum, maximum of r^3 V')
// ---------------------------------------------------------------------------
QD double dV_only(const Pot& P, double r)
{
    double V, d1, d2;
    pot_all(P, r, V, d1, d2);
    return d1;
}

// root of V' on [lo, hi] by bisection (set-up only)
QD double bisect_dV(const Pot& P, double lo, double hi)
{
    const bool inc = dV_only(P, lo) < 0.0;
    for (int it = 0; it < 400; ++it) {
        const double m = 0.5 * (lo + hi);
        if (m <= lo || m >= hi) break;
        if ((dV_only(P, m) < 0.0) == inc) lo = m; else hi = m;
    }
    return 0.5 * (lo + hi);
}

// Returns 0 on success, -1 if the potential does not have the expected shape.
QD int pair_shape(const Pot& P, Shape& Sh)
{
    Sh.rin = 0.0;
    double r = 1e-3;
    if (P.kind == BUCK) {
        // inner maximum: V' goes from + to - (geometric scan, then bisection)
        if (!(dV_only(P, r) > 0.0)) return -1;
        bool found = false;
        for (int it = 0; it < 4000 && r < kRFar; ++it) {
            const double r2 = r * 1.01;
            if (dV_only(P, r2) < 0.0) { Sh.rin = bisect_dV(P, r, r2); r = r2; found = true; break; }
            r = r2;
        }
        if (!found) return -1;
    } else {
        r = 0.05;
    }
    // minimum: V' goes from - to +
    if (!(dV_only(P, r) < 0.0)) return -1;
    bool found = false;
    for (int it = 0; it < 4000 && r < kRFar; ++it) {
        const double r2 = r * 1.01;
        if (dV_only(P, r2) > 0.0) { Sh.re = bisect_dV(P, r, r2); found = true; break; }
        r = r2;
    }
    if (!found) return -1;
    // maximum of g = r^3 V' beyond re: dg goes from + to -
    r = Sh.re * 1.0000001;
    double g, dg;
    gfun(P, r, g, dg);
    if (!(dg > 0.0)) return -1;
    found = false;
    double lo = r, hi = r;
    for (int it = 0; it < 4000 && r < kRFar; ++it) {
        const double r2 = r * 1.01;
        gfun(P, r2, g, dg);
        if (dg < 0.0) { lo = r; hi = r2; found = true; break; }
        r = r2;
    }
    if (!found) return -1;
    for (int it = 0; it < 400; ++it) {
        const double m = 0.5 * (lo + hi);
        if (m <= lo || m >= hi) break;
        gfun(P, m, g, dg);
        if (dg > 0.0) lo = m; else hi = m;
    }
    Sh.rstar = 0.5 * (lo + hi);
    gfun(P, Sh.rstar, Sh.gmax, dg);
    // single hump: dg stays negative out to kRFar (coarse check)
    for (r = hi * 1.05; r < kRFar; r *= 1.05) {
        gfun(P, r, g, dg);
        if (dg > 0.0 && g > 1e-300) return -1;
    }
    return 0;
}

}  // namespace qd
