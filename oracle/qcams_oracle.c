/*
 * qcams_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, serial, FP64 CPU implementation of the quasi-classical trajectory
 * (QCT) method of Koots & Perez-Rios, "PyQCAMS" (arXiv:2304.02731).  It is the
 * correctness reference for the HIP library and the timed CPU baseline.  Only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no source with the GPU path: constants, the Runge-Kutta
 * tableau, the random-number generator, the quadrature and every root finder
 * are written here independently.
 *
 * Everything is written for clarity, not speed: plain loops, bisection instead
 * of Newton, fine grid scans for extrema, no fusion or reordering.
 *
 * Section / equation references are to the paper:
 *   Sec. 2    Hamiltonian in Jacobi coordinates, Eq. (1)-(2); Hamilton's
 *             equations, Eq. (3)-(4).
 *   Sec. 2.1  initial conditions, Eq. (5)-(7).
 *   Sec. 2.2  bound criterion Eq. (8), j' Eq. (9), v' Eq. (10), Gaussian
 *             binning Eq. (11).
 *   Sec. 3.1  input keys (t_stop, r_stop, a_tol, r_tol; collision energy in K).
 *   Sec. 3.2  Morse / generalized Lennard-Jones / Buckingham potentials; the
 *             adaptive Runge-Kutta 5(4) integrator.
 *   Sec. 4    Morse potential Eq. (17).
 *
 * Readings of points the paper leaves open are marked "READING" below.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Physical constants (CODATA 2018).  The paper works in atomic units  */
/* and takes the collision energy in kelvin (Sec. 3.1).                */
/* ------------------------------------------------------------------ */
#define ORC_AMU_IN_ME 1822.888486209      /* unified atomic mass unit / m_e */
#define ORC_KB_IN_EH  3.1668115634556e-6  /* Boltzmann constant, E_h per K */

double orc_amu_in_me(void) { return ORC_AMU_IN_ME; }
double orc_kelvin_in_hartree(void) { return ORC_KB_IN_EH; }

/* ------------------------------------------------------------------ */
/* Input layouts (the oracle's own; mirrored by oracle/oracle.py).      */
/* ------------------------------------------------------------------ */
enum { ORC_MORSE = 0, ORC_LJ = 1, ORC_BUCK = 2 };

/* One pair interaction, Sec. 3.2:
 *   MORSE: p = {De, re, alpha}            V = De(1-exp(-alpha(r-re)))^2 - De
 *   LJ:    p = {Cn, Cm}, integers n > m   V = Cn/r^n - Cm/r^m   (READING: the
 *          printed form has the two terms swapped; the paper's own example
 *          numbers, Cm^2/(4 Cn) = De, fix this sign convention)
 *   BUCK:  p = {A, b, C6}                 V = A exp(-b r) - C6/r^6           */
typedef struct {
    int32_t kind, n, m, pad;
    double p[6];
} orc_pair;

/* masses of A, B, C in electron masses; pairs in the order AB, BC, CA
 * (AB is the initial molecule, C the colliding atom: Sec. 3.1). */
typedef struct {
    double mass[3];
    orc_pair pair[3];
} orc_system;

typedef struct {
    double R0;        /* initial atom-molecule distance scale (a0)          */
    double t_stop;    /* multiple of the collision time scale               */
    double r_stop;    /* stop when any pair distance exceeds this (a0)      */
    double atol, rtol;
    double gb_sigma;  /* width of the Gaussian binning function, Eq. (11)   */
    double h_fixed;   /* step for fixed-step mode                           */
    int32_t fixed_step;
    int32_t literal_bound; /* 1: Eq. (8) only; 0: also require r < r0        */
    int64_t max_steps;
    int32_t rk;            /* 0: Dormand-Prince 5(4); 1: Dormand-Prince 8(5,3) */
    int32_t pad;
} orc_params;

typedef struct {
    double Ec_K;      /* collision energy in kelvin */
    double b;         /* fixed impact parameter (b_mode 0) */
    double bmax;      /* maximum impact parameter (b_mode 1: b = bmax sqrt(U)) */
    int32_t b_mode, v, j, pad;
    int64_t n_traj, first_id;
    uint64_t seed;
} orc_instance;

/* Per-trajectory result record. */
typedef struct {
    double y[12];        /* rho1, rho2, P1, P2 */
    double t, tmax, rstop, e0, escale, h;
    double sample[6];    /* b, cos(theta), phi, eta, chi, weight */
    double vprime, jprime, wgb, dE_rel;
    int64_t nstep, nrej;
    int32_t status, label, vt, jt;
} orc_record;

/* trajectory status */
enum {
    ORC_RUNNING = 0, ORC_OK_RSTOP = 1, ORC_OK_TMAX = 2, ORC_FAIL_MAXSTEPS = 3,
    ORC_FAIL_NONFINITE = 4, ORC_FAIL_HMIN = 5, ORC_COLLAPSE = 6
};
/* outcome label: the product-count vector n_f = (n_q, n_r1, n_r2, n_d) of
 * Sec. 3.3, plus two bookkeeping labels.  READING: r1 = AC + B (pair CA bound),
 * r2 = BC + A (pair BC bound). */
enum { ORC_QUENCH = 0, ORC_R1 = 1, ORC_R2 = 2, ORC_DISS = 3, ORC_UNRESOLVED = 4,
       ORC_FAILED = 5 };

/* error codes */
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_EUNBOUND = -2, ORC_ENOROOT = -3 };

/* ------------------------------------------------------------------ */
/* Pair potentials and their derivatives (Sec. 3.2, Eq. (17)).          */
/* ------------------------------------------------------------------ */
void orc_potential(const orc_pair *pp, double r, double *V, double *dV)
{
    if (pp->kind == ORC_MORSE) {
        double De = pp->p[0], re = pp->p[1], a = pp->p[2];
        double e = exp(-a * (r - re));
        *V = De * (1.0 - e) * (1.0 - e) - De;
        *dV = 2.0 * De * a * e * (1.0 - e);
    } else if (pp->kind == ORC_LJ) {
        double Cn = pp->p[0], Cm = pp->p[1];
        int n = pp->n, m = pp->m;
        *V = Cn * pow(r, -n) - Cm * pow(r, -m);
        *dV = -n * Cn * pow(r, -n - 1) + m * Cm * pow(r, -m - 1);
    } else {
        double A = pp->p[0], b = pp->p[1], C6 = pp->p[2];
        *V = A * exp(-b * r) - C6 * pow(r, -6.0);
        *dV = -A * b * exp(-b * r) + 6.0 * C6 * pow(r, -7.0);
    }
}

static double pot_V(const orc_pair *pp, double r)
{
    double V, dV;
    orc_potential(pp, r, &V, &dV);
    return V;
}

static double pot_dV(const orc_pair *pp, double r)
{
    double V, dV;
    orc_potential(pp, r, &V, &dV);
    return dV;
}

/* effective potential with continuous squared angular momentum J2 (hbar = 1):
 * V(r) + J2 / (2 mu r^2), the bracket of Eq. (7), (8) and (10). */
static double veff(const orc_pair *pp, double mu, double J2, double r)
{
    return pot_V(pp, r) + J2 / (2.0 * mu * r * r);
}

static double veff_d(const orc_pair *pp, double mu, double J2, double r)
{
    return pot_dV(pp, r) - J2 / (mu * r * r * r);
}

/* plain bisection for a sign change of f on [lo, hi] */
typedef double (*orc_fn)(const orc_pair *, double, double, double, double);

static double bisect(orc_fn f, const orc_pair *pp, double mu, double J2, double c,
                     double lo, double hi)
{
    double flo = f(pp, mu, J2, c, lo);
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double fm = f(pp, mu, J2, c, mid);
        if ((fm < 0.0) == (flo < 0.0)) { lo = mid; flo = fm; }
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

static double f_veff_d(const orc_pair *pp, double mu, double J2, double c, double r)
{
    (void)c;
    return veff_d(pp, mu, J2, r);
}

static double f_veff_minus(const orc_pair *pp, double mu, double J2, double E, double r)
{
    return veff(pp, mu, J2, r) - E;
}

static double f_dV(const orc_pair *pp, double mu, double J2, double c, double r)
{
    (void)mu; (void)J2; (void)c;
    return pot_dV(pp, r);
}

/* Scan grid for the extrema of V_eff: geometric, ratio 1.002, from 0.05 a0
 * (or just outside the Buckingham inner maximum) out to ORC_RFAR. */
#define ORC_RSCAN0 0.05
#define ORC_RFAR   1.0e5
#define ORC_QSCAN  1.002

/* Inner limit of the physical region.  A Buckingham potential has a maximum
 * at short range inside which it collapses to -infinity (Sec. 3.2); this is
 * that maximum (the first + to - sign change of V').  Zero for the others. */
double orc_inner_limit(const orc_pair *pp)
{
    if (pp->kind != ORC_BUCK) return 0.0;
    double r = 1e-3, d = pot_dV(pp, r);
    if (!(d > 0.0)) return 0.0;
    while (r < ORC_RFAR) {
        double r2 = r * ORC_QSCAN, d2 = pot_dV(pp, r2);
        if (d2 < 0.0) return bisect(f_dV, pp, 0.0, 0.0, 0.0, r, r2);
        r = r2; d = d2;
    }
    return 0.0;
}

/* Extrema of V_eff(r) = V(r) + J2/(2 mu r^2) for r beyond the inner limit:
 * the well minimum r_w (first - to + sign change of V_eff') and the barrier
 * r0, "the local maximum of the effective potential" (Eq. (8)): the first
 * + to - sign change beyond r_w.  Returns 0 if there is no well; sets
 * *has_barrier = 0 when no maximum is found out to ORC_RFAR (then r0 = inf,
 * which is the J2 -> 0 limit of the barrier position). */
int orc_veff_extrema(const orc_pair *pp, double mu, double J2, double *r_w,
                     double *r_0, int *has_barrier)
{
    double rin = orc_inner_limit(pp);
    double r = fmax(rin * (1.0 + 1e-9), ORC_RSCAN0);
    double d = veff_d(pp, mu, J2, r);
    int stage = 0;           /* 0: looking for the minimum, 1: for the maximum */
    *has_barrier = 0;
    *r_0 = INFINITY;
    while (r < ORC_RFAR) {
        double r2 = r * ORC_QSCAN;
        double d2 = veff_d(pp, mu, J2, r2);
        if (stage == 0 && d < 0.0 && d2 >= 0.0) {
            *r_w = bisect(f_veff_d, pp, mu, J2, 0.0, r, r2);
            stage = 1;
        } else if (stage == 1 && d > 0.0 && d2 <= 0.0) {
            *r_0 = bisect(f_veff_d, pp, mu, J2, 0.0, r, r2);
            *has_barrier = 1;
            return 1;
        }
        r = r2; d = d2;
    }
    return stage == 1;
}

/* Classical turning points r- < r_w < r+ of V_eff at energy E, by bisection. */
int orc_turning_points(const orc_pair *pp, double mu, double J2, double E,
                       double r_w, double r_0, double *rm, double *rp)
{
    double rin = orc_inner_limit(pp);
    double lo = rin > 0.0 ? rin * (1.0 + 1e-9) : 1e-3;
    if (!(veff(pp, mu, J2, lo) > E) || !(veff(pp, mu, J2, r_w) < E)) return ORC_ENOROOT;
    double hi = isfinite(r_0) ? r_0 : ORC_RFAR;
    if (!(veff(pp, mu, J2, hi) > E)) return ORC_ENOROOT;
    *rm = bisect(f_veff_minus, pp, mu, J2, E, lo, r_w);
    *rp = bisect(f_veff_minus, pp, mu, J2, E, r_w, hi);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Gauss-Legendre nodes by Newton iteration on P_n (textbook method).   */
/* ------------------------------------------------------------------ */
#define ORC_NGL 256
static double gl_x[ORC_NGL], gl_w[ORC_NGL];
static int gl_ready = 0;

int orc_gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5)), pd = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int k = 1; k <= n; ++k) {           /* Bonnet recursion */
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
            }
            pd = n * (z * p0 - p1) / (z * z - 1.0);
            double dz = p0 / pd;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        /* recompute P_n' at the converged node for the weight */
        double p0 = 1.0, p1 = 0.0;
        for (int k = 1; k <= n; ++k) {
            double p2 = p1;
            p1 = p0;
            p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
        }
        pd = n * (z * p0 - p1) / (z * z - 1.0);
        x[i] = -z;
        w[i] = 2.0 / ((1.0 - z * z) * pd * pd);
    }
    return ORC_OK;
}

/* Radial integrals between the turning points, with the substitution
 * r = c + h sin(theta), theta in [-pi/2, pi/2], which removes the square-root
 * end-point behaviour, followed by Gauss-Legendre in theta.
 *   action: (sqrt(2 mu)/pi) int sqrt(E - V_eff) dr         (Eq. (10) + 1/2)
 *   period: sqrt(2 mu) int (E - V_eff)^(-1/2) dr            (Eq. (7))
 * The kinetic term E - V_eff(r) is a difference of nearly equal numbers at
 * the nodes next to the turning points, where the period's integrand is most
 * sensitive to it.  There it is formed as V_eff(r+-) - V_eff(r) (E =
 * V_eff(r+-) defines the turning points), i.e. as the integral of V_eff' over
 * the short interval between r and the turning point, whose length
 * h (1 - |sin theta|) = 2 h sin^2((pi/2 - |theta|)/2) is computed directly. */
#define ORC_NWALL 8
static double wall_x[ORC_NWALL], wall_w[ORC_NWALL];

static void gl_init(void)
{
    if (!gl_ready) {
        orc_gauss_legendre(ORC_NGL, gl_x, gl_w);
        orc_gauss_legendre(ORC_NWALL, wall_x, wall_w);
        gl_ready = 1;
    }
}

/* V_eff(a + len) - V_eff(a) = int_a^{a+len} V_eff'(u) du (Gauss-Legendre) */
static double veff_rise(const orc_pair *pp, double mu, double J2, double a, double len)
{
    double s = 0.0;
    for (int i = 0; i < ORC_NWALL; ++i)
        s += wall_w[i] * veff_d(pp, mu, J2, a + 0.5 * len * (1.0 + wall_x[i]));
    return 0.5 * len * s;
}

/* Node i of the rule: the factor dr/dtheta = h cos(theta) and E - V_eff(r). */
static void radial_node(const orc_pair *pp, double mu, double J2, double E, double rm,
                        double rp, int i, double *drdth, double *kin)
{
    double c = 0.5 * (rp + rm), h = 0.5 * (rp - rm);
    double x = gl_x[i];
    double u = 0.25 * M_PI * (1.0 - fabs(x));   /* (pi/2 - |theta|) / 2 */
    double d = 2.0 * h * sin(u) * sin(u);        /* distance to the nearer turning point */
    *drdth = h * sin(2.0 * u);                   /* h cos(theta) */
    if (d < 0.01 * h) {
        if (x >= 0.0) *kin = veff_rise(pp, mu, J2, rp - d, d);          /* V_eff(r+) - V_eff(r) */
        else *kin = -veff_rise(pp, mu, J2, rm, d);                       /* V_eff(r-) - V_eff(r) */
    } else {
        *kin = E - veff(pp, mu, J2, c + h * sin(0.5 * M_PI * x));
    }
}

double orc_action(const orc_pair *pp, double mu, double J2, double E, double rm, double rp)
{
    gl_init();
    double s = 0.0;
    for (int i = 0; i < ORC_NGL; ++i) {
        double dr, k;
        radial_node(pp, mu, J2, E, rm, rp, i, &dr, &k);
        if (k < 0.0) k = 0.0;
        s += gl_w[i] * sqrt(k) * dr;
    }
    s *= 0.5 * M_PI;
    return sqrt(2.0 * mu) / M_PI * s;
}

double orc_period(const orc_pair *pp, double mu, double J2, double E, double rm, double rp)
{
    gl_init();
    double s = 0.0;
    for (int i = 0; i < ORC_NGL; ++i) {
        double dr, k;
        radial_node(pp, mu, J2, E, rm, rp, i, &dr, &k);
        s += gl_w[i] * dr / sqrt(k);
    }
    s *= 0.5 * M_PI;
    return sqrt(2.0 * mu) * s;
}

/* ------------------------------------------------------------------ */
/* System geometry: reduced masses of Eq. (2) and the Jacobi map.       */
/* READING (Jacobi signs, not fixed by the paper): rho1 = r_B - r_A,    */
/* rho2 = r_C - R_cm(AB).  Pair vectors r_AB = rho1,                     */
/* r_BC = r_C - r_B = rho2 - cA rho1, r_CA = r_A - r_C = -rho2 - cB rho1 */
/* with cA = mA/(mA+mB), cB = mB/(mA+mB).                                */
/* ------------------------------------------------------------------ */
typedef struct {
    double mu12, mu123, mu_pair[3], cA, cB;
} orc_masses;

static orc_masses masses_of(const orc_system *s)
{
    orc_masses k;
    double mA = s->mass[0], mB = s->mass[1], mC = s->mass[2];
    k.mu12 = 1.0 / (1.0 / mA + 1.0 / mB);
    k.mu123 = 1.0 / (1.0 / mC + 1.0 / (mA + mB));
    k.mu_pair[0] = k.mu12;
    k.mu_pair[1] = 1.0 / (1.0 / mB + 1.0 / mC);
    k.mu_pair[2] = 1.0 / (1.0 / mC + 1.0 / mA);
    k.cA = mA / (mA + mB);
    k.cB = mB / (mA + mB);
    return k;
}

/* pair vectors and pair relative velocities from the Jacobi state */
static void pair_geometry(const orc_system *s, const double *y, double rv[3][3], double vv[3][3])
{
    orc_masses k = masses_of(s);
    for (int a = 0; a < 3; ++a) {
        double r1 = y[a], r2 = y[3 + a];
        double v1 = y[6 + a] / k.mu12, v2 = y[9 + a] / k.mu123;
        rv[0][a] = r1;
        rv[1][a] = r2 - k.cA * r1;
        rv[2][a] = -r2 - k.cB * r1;
        vv[0][a] = v1;
        vv[1][a] = v2 - k.cA * v1;
        vv[2][a] = -v2 - k.cB * v1;
    }
}

static double norm3(const double *v) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

/* Hamiltonian in Jacobi coordinates, Eq. (2). */
double orc_hamiltonian(const orc_system *s, const double *y)
{
    orc_masses k = masses_of(s);
    double rv[3][3], vv[3][3];
    pair_geometry(s, y, rv, vv);
    double T = 0.0;
    for (int a = 0; a < 3; ++a) {
        T += y[6 + a] * y[6 + a] / (2.0 * k.mu12);
        T += y[9 + a] * y[9 + a] / (2.0 * k.mu123);
    }
    double V = 0.0;
    for (int p = 0; p < 3; ++p) V += pot_V(&s->pair[p], norm3(rv[p]));
    return T + V;
}

/* Hamilton's equations, Eq. (3)-(4):  d rho_i/dt = P_i / mu_i,
 * dP_i/dt = -dV/d rho_i, with the chain rule through the pair distances. */
void orc_rhs(const orc_system *s, const double *y, double *f)
{
    orc_masses k = masses_of(s);
    double rv[3][3], vv[3][3], g[3];
    pair_geometry(s, y, rv, vv);
    for (int p = 0; p < 3; ++p) {
        double r = norm3(rv[p]);
        g[p] = pot_dV(&s->pair[p], r) / r;  /* V'(r)/r multiplies the pair vector */
    }
    for (int a = 0; a < 3; ++a) {
        f[a] = y[6 + a] / k.mu12;
        f[3 + a] = y[9 + a] / k.mu123;
        /* dV/drho1 = g_AB r_AB - cA g_BC r_BC - cB g_CA r_CA */
        f[6 + a] = -(g[0] * rv[0][a] - k.cA * g[1] * rv[1][a] - k.cB * g[2] * rv[2][a]);
        /* dV/drho2 = g_BC r_BC - g_CA r_CA */
        f[9 + a] = -(g[1] * rv[1][a] - g[2] * rv[2][a]);
    }
}

/* ------------------------------------------------------------------ */
/* Bohr-Sommerfeld levels: E_vj solves the action condition of Eq. (10) */
/* with v' = v, i.e. (sqrt(2mu)/pi) int sqrt(E - V_eff) dr = v + 1/2,   */
/* solved by bisection on E; tau_vj from Eq. (7).                       */
/* READING: the paper obtains E_int from a DVR; the build uses the      */
/* semiclassical (WKB) quantization that Eq. (10) states for v'.        */
/* out = {E, r-, r+, tau}.                                               */
/* ------------------------------------------------------------------ */
int orc_level_pair(const orc_pair *pp, double mu, int v, int j, double *out)
{
    double J2 = (double)j * (j + 1.0);
    double r_w, r_0;
    int hb;
    if (!orc_veff_extrema(pp, mu, J2, &r_w, &r_0, &hb)) return ORC_EUNBOUND;
    double Elo = veff(pp, mu, J2, r_w);
    double Ehi = hb ? veff(pp, mu, J2, r_0) : 0.0;
    double target = v + 0.5;
    double rm, rp;
    /* top of the well: the action there must exceed v + 1/2 */
    double Etop = Ehi - 1e-13 * fabs(Ehi - Elo);
    if (orc_turning_points(pp, mu, J2, Etop, r_w, r_0, &rm, &rp) != ORC_OK) return ORC_EUNBOUND;
    if (orc_action(pp, mu, J2, Etop, rm, rp) <= target) return ORC_EUNBOUND;
    double lo = Elo, hi = Etop;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (orc_turning_points(pp, mu, J2, mid, r_w, r_0, &rm, &rp) != ORC_OK) { lo = mid; continue; }
        if (orc_action(pp, mu, J2, mid, rm, rp) < target) lo = mid; else hi = mid;
    }
    double E = 0.5 * (lo + hi);
    if (orc_turning_points(pp, mu, J2, E, r_w, r_0, &rm, &rp) != ORC_OK) return ORC_ENOROOT;
    out[0] = E;
    out[1] = rm;
    out[2] = rp;
    out[3] = orc_period(pp, mu, J2, E, rm, rp);
    return ORC_OK;
}

int orc_level(const orc_system *s, int v, int j, double *out)
{
    orc_masses k = masses_of(s);
    return orc_level_pair(&s->pair[0], k.mu12, v, j, out);
}

/* ------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), from its          */
/* published definition.  READING: the paper only says "seed"; the      */
/* build uses this counter-based generator, key = (seed, 0),            */
/* counter = (trajectory id, block, 0, 0), uniform = (u >> 11) * 2^-53. */
/* ------------------------------------------------------------------ */
void orc_philox4x64_10(const uint64_t *ctr_in, const uint64_t *key_in, uint64_t *out)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double u01(uint64_t u) { return (double)(u >> 11) * (1.0 / 9007199254740992.0); }

/* the six uniforms of one trajectory: b, cos(theta), phi, eta (block 0),
 * chi and the proposal cell (block 1) */
void orc_uniforms(uint64_t seed, int64_t id, double *u)
{
    uint64_t key[2] = {seed, 0}, ctr[4] = {(uint64_t)id, 0, 0, 0}, out[4];
    orc_philox4x64_10(ctr, key, out);
    for (int i = 0; i < 4; ++i) u[i] = u01(out[i]);
    ctr[1] = 1;
    orc_philox4x64_10(ctr, key, out);
    u[4] = u01(out[0]);
    u[5] = u01(out[1]);
}

/* Importance-sampling proposal over cells of (b^2, chi, cos theta): 32 x 16
 * x 16 cells of equal measure under the uniform sampling of Sec. 2.3, index
 * (ib*16 + ichi)*16 + icos, cell probabilities q (any positive scale).  A
 * draw picks the first cell whose running sum of q/sum(q) exceeds the cell
 * uniform and a uniform point inside it; its weight is (1/K)/(q_k/sum q),
 * which keeps the Monte Carlo estimates of Eq. (13) unbiased. */
#define ORC_CELLS 8192
static void proposal_draw(const double *q, const double *u, double bmax, double *b,
                          double *cth, double *chi, double *w)
{
    double tot = 0.0, run = 0.0;
    for (int i = 0; i < ORC_CELLS; ++i) tot += q[i];
    int k = ORC_CELLS - 1;
    for (int i = 0; i < ORC_CELLS; ++i) {
        run += q[i];
        if (run / tot > u[5]) { k = i; break; }
    }
    int ib = k / 256, ichi = (k / 16) % 16, ic = k % 16;
    *b = bmax * sqrt((ib + u[0]) / 32.0);
    *cth = -1.0 + (ic + u[1]) * (2.0 / 16.0);
    *chi = (ichi + u[4]) / 16.0;
    *w = (1.0 / ORC_CELLS) / (q[k] / tot);
}

/* ------------------------------------------------------------------ */
/* Initial conditions, Sec. 2.1.                                        */
/* level = {E_vj, r-, r+, tau}.  Outputs the 12-vector y and            */
/* aux = {t, tmax, rstop_eff, e0, escale, h}, sample = {b, cos(theta),   */
/* phi, eta, chi, weight}.                                              */
/* ------------------------------------------------------------------ */
int orc_init_q(const orc_system *s, const orc_params *prm, const orc_instance *in,
               const double *level, int64_t id, double *y, double *aux, double *sample,
               const double *prop_q)
{
    orc_masses k = masses_of(s);
    double u[6];
    orc_uniforms(in->seed, id, u);
    /* READING: uniform measure d(Omega) = sin(theta) dtheta dphi deta dchi
     * (Sec. 2.3): cos(theta) in [-1,1), phi, eta in [0, 2pi), chi in [0,1).
     * Impact parameter fixed, or uniform in area up to bmax. */
    double b = in->b_mode == 1 ? in->bmax * sqrt(u[0]) : in->b;
    double cth = 2.0 * u[1] - 1.0;
    double phi = 2.0 * M_PI * u[2];
    double eta = 2.0 * M_PI * u[3];
    double chi = u[4];
    double wgt = 1.0;
    if (in->b_mode == 2) {
        if (!prop_q) return ORC_EINVAL;
        proposal_draw(prop_q, u, in->bmax, &b, &cth, &chi, &wgt);
    }
    double sth = sqrt(1.0 - cth * cth);
    double rp = level[2], tau = level[3];
    double jj = (double)in->j;
    /* molecule at its outer turning point, momentum perpendicular, Eq. (5) */
    double P1 = sqrt(jj * (jj + 1.0)) / rp;
    y[0] = rp * sth * cos(phi);
    y[1] = rp * sth * sin(phi);
    y[2] = rp * cth;
    y[6] = P1 * (sin(phi) * cos(eta) - cth * cos(phi) * sin(eta));
    y[7] = P1 * (-cos(phi) * cos(eta) - cth * sin(phi) * sin(eta));
    y[8] = P1 * (sth * sin(eta));
    /* atom: collision momentum along +z, impact parameter along +y; the
     * vibrational phase enters through the distance, Eq. (6). */
    double Ec = in->Ec_K * ORC_KB_IN_EH;
    double P2 = sqrt(2.0 * k.mu123 * Ec);
    double R = prm->R0 + chi * P2 * tau / k.mu123;
    if (!(b < R)) return ORC_EINVAL;
    y[3] = 0.0;
    y[4] = b;
    y[5] = -sqrt(R * R - b * b);
    y[9] = 0.0;
    y[10] = 0.0;
    y[11] = P2;
    /* READING: t_max = t_stop * (d / v_c) with d = R and v_c = P2/mu123
     * (Sec. 3.1); the distance cut-off is shifted by the phase offset. */
    double vc = P2 / k.mu123;
    double e0 = orc_hamiltonian(s, y);
    aux[0] = 0.0;
    aux[1] = prm->t_stop * R / vc;
    aux[2] = prm->r_stop + (R - prm->R0);
    aux[3] = e0;
    aux[4] = fmax(fabs(e0), fabs(level[0]));
    aux[5] = 0.0;
    sample[0] = b; sample[1] = cth; sample[2] = phi; sample[3] = eta; sample[4] = chi;
    sample[5] = wgt;
    return ORC_OK;
}

int orc_init(const orc_system *s, const orc_params *prm, const orc_instance *in,
             const double *level, int64_t id, double *y, double *aux, double *sample)
{
    return orc_init_q(s, prm, in, level, id, y, aux, sample, 0);
}

/* ------------------------------------------------------------------ */
/* Dormand-Prince 5(4) (Dormand & Prince 1980), the adaptive RK5(4) of  */
/* Sec. 3.2.  Tableau written from the published coefficients.          */
/* ------------------------------------------------------------------ */
static const double DP_C[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
static const double DP_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84},
};
static const double DP_B[7] = {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84, 0};
static const double DP_BH[7] = {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640,
                                -92097.0 / 339200, 187.0 / 2100, 1.0 / 40};

void orc_dopri5_tableau(double *c, double *a, double *b, double *bh)
{
    for (int i = 0; i < 7; ++i) {
        c[i] = DP_C[i]; b[i] = DP_B[i]; bh[i] = DP_BH[i];
        for (int j = 0; j < 7; ++j) a[7 * i + j] = j < 6 ? DP_A[i][j] : 0.0;
    }
}

/* one DOPRI5 step from (y, k1 = f(y)) with step h: ynew, k7 = f(ynew), and
 * the embedded error estimate e = h sum (b - bhat) k. */
static void dp_step(const orc_system *s, const double *y, const double *k1, double h,
                    double *ynew, double *k7, double *err)
{
    double k[7][12], yt[12];
    memcpy(k[0], k1, sizeof(double) * 12);
    for (int st = 1; st < 7; ++st) {
        for (int i = 0; i < 12; ++i) {
            double acc = 0.0;
            for (int l = 0; l < st; ++l) acc += DP_A[st][l] * k[l][i];
            yt[i] = y[i] + h * acc;
        }
        orc_rhs(s, yt, k[st]);
        if (st == 6) memcpy(ynew, yt, sizeof(double) * 12);
    }
    memcpy(k7, k[6], sizeof(double) * 12);
    for (int i = 0; i < 12; ++i) {
        double e = 0.0;
        for (int l = 0; l < 7; ++l) e += (DP_B[l] - DP_BH[l]) * k[l][i];
        err[i] = h * e;
    }
}

/* Dormand-Prince 8(5,3) ("DOP853", Hairer-Norsett-Wanner I, Sec. II.10):
 * 12 stages, 8th-order solution, error estimated from a 5th-order and a
 * 3rd-order embedded combination that also use f(y_new) (stage 13).  The
 * published coefficients are handed in once by the caller. */
static double D8_A[12][12], D8_B[12], D8_C[12], D8_E3[13], D8_E5[13];
static int d8_ready = 0;

void orc_set_dop853(const double *A, const double *B, const double *C, const double *E3,
                    const double *E5)
{
    for (int i = 0; i < 12; ++i) {
        for (int j = 0; j < 12; ++j) D8_A[i][j] = A[12 * i + j];
        D8_B[i] = B[i];
        D8_C[i] = C[i];
    }
    for (int i = 0; i < 13; ++i) { D8_E3[i] = E3[i]; D8_E5[i] = E5[i]; }
    d8_ready = 1;
}

/* one DOP853 step: ynew, k13 = f(ynew) and the combined error norm
 * err = |e5|^2 / sqrt((|e5|^2 + 0.01 |e3|^2) n) over the scaled components */
static double d8_step(const orc_system *s, const double *y, const double *k1, double h,
                      double atol, double rtol, double *ynew, double *k13)
{
    double k[13][12], yt[12];
    memcpy(k[0], k1, sizeof(double) * 12);
    for (int st = 1; st < 12; ++st) {
        for (int i = 0; i < 12; ++i) {
            double acc = 0.0;
            for (int l = 0; l < st; ++l) acc += D8_A[st][l] * k[l][i];
            yt[i] = y[i] + h * acc;
        }
        orc_rhs(s, yt, k[st]);
    }
    for (int i = 0; i < 12; ++i) {
        double acc = 0.0;
        for (int l = 0; l < 12; ++l) acc += D8_B[l] * k[l][i];
        ynew[i] = y[i] + h * acc;
    }
    orc_rhs(s, ynew, k[12]);
    memcpy(k13, k[12], sizeof(double) * 12);
    double n5 = 0.0, n3 = 0.0;
    for (int i = 0; i < 12; ++i) {
        double e5 = 0.0, e3 = 0.0;
        for (int l = 0; l < 13; ++l) { e5 += D8_E5[l] * k[l][i]; e3 += D8_E3[l] * k[l][i]; }
        double sc = atol + rtol * fmax(fabs(y[i]), fabs(ynew[i]));
        n5 += (h * e5 / sc) * (h * e5 / sc);
        n3 += (h * e3 / sc) * (h * e3 / sc);
    }
    if (n5 == 0.0 && n3 == 0.0) return 0.0;
    return n5 / sqrt((n5 + 0.01 * n3) * 12.0);
}

/* RMS error norm, Hairer-Norsett-Wanner I, Sec. II.4 */
static double err_norm(const double *y, const double *ynew, const double *e, double atol, double rtol)
{
    double s = 0.0;
    for (int i = 0; i < 12; ++i) {
        double sc = atol + rtol * fmax(fabs(y[i]), fabs(ynew[i]));
        s += (e[i] / sc) * (e[i] / sc);
    }
    return sqrt(s / 12.0);
}

/* starting step, Hairer-Norsett-Wanner I, Sec. II.4 */
static double initial_step(const orc_system *s, const double *y, const double *f0,
                           double atol, double rtol, double span, double order)
{
    double d0 = 0.0, d1 = 0.0, y1[12], f1[12], d2 = 0.0;
    for (int i = 0; i < 12; ++i) {
        double sc = atol + rtol * fabs(y[i]);
        d0 += (y[i] / sc) * (y[i] / sc);
        d1 += (f0[i] / sc) * (f0[i] / sc);
    }
    d0 = sqrt(d0 / 12.0);
    d1 = sqrt(d1 / 12.0);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    if (h0 > span) h0 = span;
    for (int i = 0; i < 12; ++i) y1[i] = y[i] + h0 * f0[i];
    orc_rhs(s, y1, f1);
    for (int i = 0; i < 12; ++i) {
        double sc = atol + rtol * fabs(y[i]);
        d2 += ((f1[i] - f0[i]) / sc) * ((f1[i] - f0[i]) / sc);
    }
    d2 = sqrt(d2 / 12.0) / h0;
    double dm = fmax(d1, d2);
    double h1 = dm <= 1e-15 ? fmax(1e-6, h0 * 1e-3) : pow(0.01 / dm, 1.0 / order);
    double h = fmin(100.0 * h0, h1);
    return fmin(h, span);
}

/* Error norm of one adaptive trial step of size h from state y (the
 * integrator of prm->rk), as the adaptive loop below evaluates it. */
double orc_trial_error(const orc_system *s, const orc_params *prm, const double *y, double h)
{
    double f0[12], ynew[12], k7[12], e[12];
    orc_rhs(s, y, f0);
    if (prm->rk == 1) {
        if (!d8_ready) return NAN;
        return d8_step(s, y, f0, h, prm->atol, prm->rtol, ynew, k7);
    }
    dp_step(s, y, f0, h, ynew, k7, e);
    return err_norm(y, ynew, e, prm->atol, prm->rtol);
}

/* Buckingham collapse radius of each pair (0 if none). */
static void collapse_radii(const orc_system *s, double *rb)
{
    for (int p = 0; p < 3; ++p) rb[p] = orc_inner_limit(&s->pair[p]);
}

/* READING of the stop rules (Sec. 3.1): stop after the first accepted step at
 * which the largest pair distance exceeds rstop_eff (distances compared as
 * squares), or when t reaches t_max; also stop on step-count exhaustion,
 * non-finite state, step-size underflow, or a pair falling inside a
 * Buckingham inner maximum.  Step-size control: RMS error norm, accept if
 * err <= 1, factor min(10, max(0.2, 0.9 err^(-1/5))), no increase right after
 * a rejection, h_min = 1e-12 t_max. */
int orc_propagate_log(const orc_system *s, const orc_params *prm, double *y, double *aux,
                      int64_t *nstep, int64_t *nrej, double *log, int64_t log_cap,
                      int64_t *log_n);

int orc_propagate(const orc_system *s, const orc_params *prm, double *y, double *aux,
                  int64_t *nstep, int64_t *nrej)
{
    return orc_propagate_log(s, prm, y, aux, nstep, nrej, 0, 0, 0);
}

/* orc_propagate with a record of every trial step (test diagnostics):
 * log[16 k + 0..3] = (t, trial step size, error norm, 1 if accepted) and
 * log[16 k + 4..15] = the state the trial starts from, for the first
 * log_cap trials; *log_n = the number of trials made. */
int orc_propagate_log(const orc_system *s, const orc_params *prm, double *y, double *aux,
                      int64_t *nstep, int64_t *nrej, double *log, int64_t log_cap,
                      int64_t *log_n)
{
    int64_t ntrial = 0;
    double f0[12], ynew[12], k7[12], e[12], rb[3];
    collapse_radii(s, rb);
    double t = aux[0], tmax = aux[1], rs = aux[2], h = aux[5];
    const int d8 = prm->rk == 1;
    if (d8 && !d8_ready) return ORC_FAIL_NONFINITE;
    /* step-size exponent 1/(q+1), q the order of the error estimate */
    const double expo = d8 ? 1.0 / 8.0 : 1.0 / 5.0;
    orc_rhs(s, y, f0);
    if (prm->fixed_step) h = prm->h_fixed;
    else if (!(h > 0.0)) h = initial_step(s, y, f0, prm->atol, prm->rtol, tmax - t, d8 ? 8.0 : 5.0);
    double hmin = 1e-12 * tmax;
    int status = ORC_RUNNING, last_rejected = 0;
    if (t >= tmax) status = ORC_OK_TMAX;
    while (status == ORC_RUNNING) {
        if (*nstep >= prm->max_steps) { status = ORC_FAIL_MAXSTEPS; break; }
        double hs = fmin(h, tmax - t);
        double err;
        if (d8) {
            err = d8_step(s, y, f0, hs, prm->atol, prm->rtol, ynew, k7);
        } else {
            dp_step(s, y, f0, hs, ynew, k7, e);
            err = err_norm(y, ynew, e, prm->atol, prm->rtol);
        }
        if (prm->fixed_step) err = 0.0;
        if (!isfinite(err)) err = INFINITY;
        if (log && ntrial < log_cap) {
            double *rec = log + 16 * ntrial;
            rec[0] = t;
            rec[1] = hs;
            rec[2] = err;
            rec[3] = err <= 1.0 ? 1.0 : 0.0;
            memcpy(rec + 4, y, sizeof y[0] * 12);
        }
        ++ntrial;
        if (err <= 1.0) {
            t = (hs == tmax - t) ? tmax : t + hs;
            memcpy(y, ynew, sizeof y[0] * 12);
            memcpy(f0, k7, sizeof f0);
            *nstep += 1;
            int finite = 1;
            for (int i = 0; i < 12; ++i) finite &= isfinite(y[i]);
            double rv[3][3], vv[3][3], rmax2 = 0.0;
            pair_geometry(s, y, rv, vv);
            int collapsed = 0;
            for (int p = 0; p < 3; ++p) {
                double r2 = rv[p][0] * rv[p][0] + rv[p][1] * rv[p][1] + rv[p][2] * rv[p][2];
                if (r2 > rmax2) rmax2 = r2;
                if (r2 < rb[p] * rb[p]) collapsed = 1;
            }
            if (!finite) status = ORC_FAIL_NONFINITE;
            else if (collapsed) status = ORC_COLLAPSE;
            else if (rmax2 > rs * rs) status = ORC_OK_RSTOP;
            else if (t >= tmax) status = ORC_OK_TMAX;
            if (!prm->fixed_step) {
                double fac = err == 0.0 ? 10.0 : fmin(10.0, fmax(0.2, 0.9 * pow(err, -expo)));
                if (last_rejected && fac > 1.0) fac = 1.0;
                h = hs * fac;
            }
            last_rejected = 0;
        } else {
            *nrej += 1;
            h = hs * fmax(0.2, 0.9 * pow(err, -expo));
            last_rejected = 1;
        }
        if (status == ORC_RUNNING && !prm->fixed_step && h < hmin) status = ORC_FAIL_HMIN;
    }
    aux[0] = t;
    aux[5] = h;
    if (log_n) *log_n = ntrial;
    return status;
}

/* ------------------------------------------------------------------ */
/* Product classification, Sec. 2.2.                                    */
/* ------------------------------------------------------------------ */
/* Eq. (8) for one pair, with continuous J2 = j'(j'+1).  READING: r0 is the
 * outer maximum of V_eff beyond its well; with no well the pair is unbound;
 * with no maximum (J2 -> 0) the threshold is 0; unless literal_bound is set
 * the pair must also lie inside the barrier (r < r0). */
int orc_pair_bound(const orc_pair *pp, double mu, double J2, double E, double r,
                   int literal, double *r_w_out, double *r_0_out)
{
    double r_w, r_0;
    int hb;
    if (!orc_veff_extrema(pp, mu, J2, &r_w, &r_0, &hb)) return 0;
    double thr = (hb && J2 > 0.0) ? veff(pp, mu, J2, r_0) : 0.0;
    if (!hb) r_0 = INFINITY;
    if (r_w_out) *r_w_out = r_w;
    if (r_0_out) *r_0_out = r_0;
    if (!(E < thr)) return 0;
    if (!literal && !(r < r_0)) return 0;
    return 1;
}

/* Gaussian binning weight, Eq. (11), against the nearest integer vt */
double orc_gb_weight(double vprime, double sigma, int *vt)
{
    double n = floor(vprime + 0.5);
    *vt = (int)n;
    double d = vprime - n;
    return exp(-d * d / (2.0 * sigma * sigma)) / (sigma * sqrt(2.0 * M_PI));
}

/* Final-state analysis of one trajectory: label, v', j', (vt, jt) and the
 * Gaussian weight; s_f = (0, 0, 0) when no single pair is bound (Sec. 3.3). */
int orc_classify(const orc_system *s, const orc_params *prm, const double *y,
                 int *label, int *vt, int *jt, double *vprime, double *jprime, double *wgb,
                 double *pair_E, double *pair_J2)
{
    orc_masses k = masses_of(s);
    double rv[3][3], vv[3][3], E[3], J2[3], r[3];
    int bound[3], nb = 0;
    pair_geometry(s, y, rv, vv);
    for (int p = 0; p < 3; ++p) {
        double mu = k.mu_pair[p];
        r[p] = norm3(rv[p]);
        double v2 = vv[p][0] * vv[p][0] + vv[p][1] * vv[p][1] + vv[p][2] * vv[p][2];
        E[p] = 0.5 * mu * v2 + pot_V(&s->pair[p], r[p]);
        double Lx = rv[p][1] * vv[p][2] - rv[p][2] * vv[p][1];
        double Ly = rv[p][2] * vv[p][0] - rv[p][0] * vv[p][2];
        double Lz = rv[p][0] * vv[p][1] - rv[p][1] * vv[p][0];
        J2[p] = mu * mu * (Lx * Lx + Ly * Ly + Lz * Lz);
        bound[p] = orc_pair_bound(&s->pair[p], mu, J2[p], E[p], r[p], prm->literal_bound, 0, 0);
        nb += bound[p];
        if (pair_E) pair_E[p] = E[p];
        if (pair_J2) pair_J2[p] = J2[p];
    }
    *vt = 0; *jt = 0; *vprime = 0.0; *jprime = 0.0; *wgb = 0.0;
    if (nb == 0) { *label = ORC_DISS; return ORC_OK; }
    if (nb > 1) { *label = ORC_UNRESOLVED; return ORC_OK; }
    int p = bound[0] ? 0 : (bound[2] ? 2 : 1);
    *label = p == 0 ? ORC_QUENCH : (p == 2 ? ORC_R1 : ORC_R2);
    double mu = k.mu_pair[p];
    /* rotational number, Eq. (9) */
    *jprime = -0.5 + 0.5 * sqrt(1.0 + 4.0 * J2[p]);
    *jt = (int)floor(*jprime + 0.5);
    /* vibrational number, Eq. (10), with E'_int = the pair energy */
    double r_w, r_0, rm, rp;
    orc_pair_bound(&s->pair[p], mu, J2[p], E[p], r[p], 1, &r_w, &r_0);
    if (orc_turning_points(&s->pair[p], mu, J2[p], E[p], r_w, r_0, &rm, &rp) != ORC_OK) {
        *label = ORC_UNRESOLVED;
        *jt = 0; *jprime = 0.0;
        return ORC_OK;
    }
    *vprime = orc_action(&s->pair[p], mu, J2[p], E[p], rm, rp) - 0.5;
    *wgb = orc_gb_weight(*vprime, prm->gb_sigma, vt);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* One full trajectory and a batch driver.                              */
/* ------------------------------------------------------------------ */
int orc_run_one(const orc_system *s, const orc_params *prm, const orc_instance *in,
                const double *level, int64_t id, orc_record *rec, const double *prop_q)
{
    memset(rec, 0, sizeof *rec);
    double aux[6];
    int rc = orc_init_q(s, prm, in, level, id, rec->y, aux, rec->sample, prop_q);
    if (rc != ORC_OK) return rc;
    rec->status = orc_propagate(s, prm, rec->y, aux, &rec->nstep, &rec->nrej);
    rec->t = aux[0]; rec->tmax = aux[1]; rec->rstop = aux[2]; rec->e0 = aux[3];
    rec->escale = aux[4]; rec->h = aux[5];
    rec->dE_rel = (orc_hamiltonian(s, rec->y) - rec->e0) / rec->escale;
    if (rec->status == ORC_OK_RSTOP || rec->status == ORC_OK_TMAX) {
        orc_classify(s, prm, rec->y, &rec->label, &rec->vt, &rec->jt, &rec->vprime,
                     &rec->jprime, &rec->wgb, 0, 0);
    } else {
        rec->label = ORC_FAILED;
    }
    return ORC_OK;
}

/* Run trajectories ids[0..n) of instance `in` (level precomputed). */
int orc_run_batch(const orc_system *s, const orc_params *prm, const orc_instance *in,
                  const double *level, const int64_t *ids, int64_t n, orc_record *out,
                  const double *prop_q)
{
    for (int64_t i = 0; i < n; ++i) {
        int rc = orc_run_one(s, prm, in, level, ids[i], &out[i], prop_q);
        if (rc != ORC_OK) return rc;
    }
    return ORC_OK;
}
