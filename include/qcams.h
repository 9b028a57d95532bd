/*
 * qcams.h -- C ABI of the MI355X (gfx950) quasi-classical trajectory library.
 *
 * The calls follow the problem statement of Koots & Perez-Rios, "PyQCAMS"
 * (arXiv:2304.02731): an atom C collides with a diatomic molecule AB on a
 * pairwise-additive surface (Morse, generalized Lennard-Jones or Buckingham
 * pairs, Sec. 3.2); each trajectory starts from a Bohr-Sommerfeld (v, j) state
 * with random orientation and vibrational phase (Sec. 2.1), is integrated with
 * an adaptive Dormand-Prince RK5(4) (Sec. 2, Eq. (3)-(4); Sec. 3.2), and ends
 * with classification into quench / reaction / dissociation and Gaussian
 * binning of the product's (v', j') (Sec. 2.2); cross sections, Monte Carlo
 * errors and rates follow (Sec. 2.3 Eq. (12)-(16); Sec. 4 Eq. (18)-(19)).
 *
 * Conventions for every call:
 *  - Units: atomic units (hbar = m_e = a0 = E_h = 1), except collision
 *    energies, which are given in kelvin (as the paper's input file does).
 *    Masses are in electron masses or, with qcams_system.mass_unit =
 *    QCAMS_MASS_AMU, in unified atomic mass units (converted by the library).
 *  - Return value: QCAMS_OK (0) or a negative QCAMS_E* code; qcams_last_error
 *    gives a message.  No exception or abort crosses the ABI.  Problems of a
 *    single trajectory are reported in its status / label, never as a call
 *    error.
 *  - Memory: pointers documented "device" are device memory owned by the
 *    caller; they must stay valid until the work queued on `stream` has
 *    finished.  The library never frees or keeps them.  "host" pointers are
 *    read (or written) before the call returns.  The library owns only the
 *    context.
 *  - Streams: `stream` is a hipStream_t (NULL = the default stream).  Calls
 *    marked "async" only enqueue kernels on it; calls marked "sync" block.
 *    A context's device work tables (the persistent run's work lists and
 *    wave-step count, the reduction's per-chunk partial sums) are shared by
 *    its calls: qcams_run and qcams_cross_sections calls on one context must
 *    not overlap on different streams (one stream per context, or a context
 *    per stream); qcams_set_instances must not overlap queued work of the
 *    context either.
 *  - Determinism: every result is a pure function of (system, params,
 *    instances, seed, trajectory id); integer results are bit-reproducible
 *    and floating-point reductions use a fixed order.
 *  - Structure-of-arrays: per-trajectory arrays are laid out field-major with
 *    a leading dimension `ld` >= the number of trajectories (element i of
 *    field f at [f * ld + i]).
 */
#ifndef QCAMS_H
#define QCAMS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---- */
#define QCAMS_OK 0
#define QCAMS_EINVAL (-1)   /* bad argument */
#define QCAMS_EUNBOUND (-2) /* a requested (v, j) level is not bound */
#define QCAMS_ENOROOT (-3)  /* a level / shape root could not be bracketed */
#define QCAMS_EHIP (-4)     /* a HIP runtime call failed */
#define QCAMS_ENOMEM (-5)   /* device allocation failed */

/* ---- pair potentials (Sec. 3.2; Eq. (17)) ---- */
#define QCAMS_MORSE 0 /* V = De (1 - exp(-alpha (r - re)))^2 - De;  p = {De, re, alpha} */
#define QCAMS_LJ 1    /* V = Cn r^-n - Cm r^-m, integers n > m >= 3;  p = {Cn, Cm} */
#define QCAMS_BUCK 2  /* V = A exp(-b r) - C6 r^-6;  p = {A, b, C6} */
/* Input forms, converted by the library (qcams_system_resolve):
 * QCAMS_MORSE_WE: the Morse pair by its harmonic frequency, as the paper's
 *   input file gives it (keys de, re, we):  p = {De, re, w_e};
 *   alpha = w_e sqrt(mu / (2 De)) with mu the pair's reduced mass.
 * QCAMS_LJ_EPS: the LJ pair by the depth eps and position r_m of its
 *   minimum, exponents n > m >= 3:  p = {eps, r_m};
 *   Cn = eps m r_m^n / (n - m), Cm = eps n r_m^m / (n - m). */
#define QCAMS_MORSE_WE 3
#define QCAMS_LJ_EPS 4

/* ---- mass units ---- */
#define QCAMS_MASS_ME 0  /* electron masses */
#define QCAMS_MASS_AMU 1 /* unified atomic mass units: 1 u = 1822.888486209 m_e (CODATA 2018) */

/* ---- impact-parameter sampling ---- */
#define QCAMS_B_FIXED 0    /* every trajectory at b */
#define QCAMS_B_AREA 1     /* b = bmax sqrt(U): uniform over the disc of radius bmax */
#define QCAMS_B_PROPOSAL 2 /* (b^2, chi, cos theta) from the installed proposal, with weights */

/* ---- trajectory status ---- */
#define QCAMS_RUNNING 0
#define QCAMS_OK_RSTOP 1        /* a pair distance exceeded r_stop (shifted, see below) */
#define QCAMS_OK_TMAX 2         /* t reached t_max */
#define QCAMS_FAIL_MAXSTEPS 3   /* max_steps accepted steps without stopping */
#define QCAMS_FAIL_NONFINITE 4  /* non-finite state */
#define QCAMS_FAIL_HMIN 5       /* step size fell below 1e-12 t_max */
#define QCAMS_COLLAPSE 6        /* a Buckingham pair fell inside its inner maximum */

/* ---- outcome labels: the product-count vector (n_q, n_r1, n_r2, n_d), Sec. 3.3 ---- */
#define QCAMS_QUENCH 0     /* AB bound:  AB(v') + C  */
#define QCAMS_R1 1         /* CA bound:  AC + B      */
#define QCAMS_R2 2         /* BC bound:  BC + A      */
#define QCAMS_DISS 3       /* no pair bound: A + B + C */
#define QCAMS_UNRESOLVED 4 /* more than one pair bound (the paper requires exactly one) */
#define QCAMS_FAILED 5     /* the trajectory did not end with OK_RSTOP / OK_TMAX */

typedef struct {
    int32_t kind; /* QCAMS_MORSE / QCAMS_LJ / QCAMS_BUCK / QCAMS_MORSE_WE / QCAMS_LJ_EPS */
    int32_t n, m; /* LJ exponents (n > m), ignored otherwise */
    int32_t pad;
    double p[6];  /* see the kind's comment; unused entries ignored */
} qcams_pair;

typedef struct {
    double mass[3];     /* mA, mB, mC in mass_unit; AB is the molecule */
    qcams_pair pair[3]; /* AB, BC, CA */
    int32_t mass_unit;  /* QCAMS_MASS_ME (0) or QCAMS_MASS_AMU */
    int32_t pad;
} qcams_system;

typedef struct {
    double R0;       /* distance of the atom from the molecule before the phase shift (a0), Eq. (6) */
    double t_stop;   /* t_max = t_stop * R / v_c, v_c = collision speed (Sec. 3.1) */
    double r_stop;   /* stop when a pair distance exceeds r_stop + (R - R0) (Sec. 3.1) */
    double atol;     /* absolute tolerance of the RK5(4) error control */
    double rtol;     /* relative tolerance */
    double gb_sigma; /* Gaussian-binning width of Eq. (11) */
    double h_fixed;  /* step of fixed-step mode */
    int32_t fixed_step;    /* 1: no error control, step h_fixed */
    int32_t literal_bound; /* 1: Eq. (8) alone; 0: also require the pair inside its barrier */
    int64_t max_steps;     /* accepted steps per trajectory, 1 .. 2^31-1 */
    int32_t rk;            /* QCAMS_RK_DOPRI5 (the paper's RK45) or QCAMS_RK_DOP853 */
    int32_t pad;
} qcams_params;

/* ---- Runge-Kutta variants of the adaptive integrator ---- */
#define QCAMS_RK_DOPRI5 0 /* Dormand-Prince 5(4): controller exponent 1/5 */
#define QCAMS_RK_DOP853 1 /* Dormand-Prince 8(5,3): exponent 1/8, Hairer's combined error */

typedef struct {
    double Ec_K;       /* collision energy (kelvin) */
    double b;          /* impact parameter for QCAMS_B_FIXED (a0) */
    double bmax;       /* maximum impact parameter for QCAMS_B_AREA (a0) */
    int32_t b_mode;    /* QCAMS_B_FIXED / QCAMS_B_AREA */
    int32_t v, j;      /* initial rovibrational level of AB */
    int32_t pad;
    int64_t n_traj;    /* trajectories of this instance */
    int64_t first_id;  /* global id of its first trajectory; ids are contiguous */
    uint64_t seed;     /* random stream key (Philox4x64-10, key = (seed, 0)) */
} qcams_instance;

/* Per-trajectory double fields of the state, [QCAMS_NF][ld] */
#define QCAMS_NF 18
#define QCAMS_F_X 0       /* 0..5:  rho1 (3), rho2 (3) -- Jacobi vectors (Sec. 2) */
#define QCAMS_F_P 6       /* 6..11: P1 (3), P2 (3) -- conjugate momenta */
#define QCAMS_F_T 12      /* time */
#define QCAMS_F_TMAX 13   /* t_max */
#define QCAMS_F_RSTOP 14  /* effective r_stop */
#define QCAMS_F_E0 15     /* initial total energy H(0) */
#define QCAMS_F_ESCALE 16 /* energy scale max(|H(0)|, |E_vj|) for the conservation check */
#define QCAMS_F_H 17      /* next step size (<= 0: choose the starting step) */

typedef struct {
    double *d;        /* device [QCAMS_NF][ld] */
    int32_t *nstep;   /* device [ld] accepted steps */
    int32_t *nrej;    /* device [ld] rejected steps */
    uint8_t *status;  /* device [ld] QCAMS_RUNNING / QCAMS_OK_* / QCAMS_FAIL_* */
    int64_t ld;
} qcams_state;

/* Per-trajectory sample fields, [QCAMS_NS][ld]: b, cos(theta), phi, eta, chi, weight */
#define QCAMS_NS 6

/* Per-trajectory outcome.  d = [4][ld]: v', j' (Eq. (9)-(10)), Gaussian weight
 * W (Eq. (11)), (H(t_f) - H(0)) / escale.  (vt, jt, W) = (0, 0, 0) unless
 * exactly one pair is bound (the paper's s_f for dissociation, Sec. 3.3). */
typedef struct {
    uint8_t *label;   /* device [ld] QCAMS_QUENCH .. QCAMS_FAILED */
    int16_t *vt;      /* device [ld] nearest integer of v' */
    int16_t *jt;      /* device [ld] nearest integer of j' */
    double *d;        /* device [4][ld] */
    int64_t ld;
} qcams_outcome;

/* Per-instance results, rows of QCAMS_XS_STRIDE doubles:
 *   [0] N, [1..6] counts per label, [7..10] P_x = (1/N) sum w 1[x] for
 *   x = q, r1, r2, d (Eq. (13)), [11..14] its Monte Carlo error (Eq. (16)
 *   when w = 1), [15..18] sigma_x, [19..22] error of sigma_x, [23..26] rate
 *   k_x = sigma_x sqrt(2 E_c / mu_123) (Eq. (19)), [27] total weight W of
 *   Eq. (15), [28] sum w, [29] sum w^2.  sigma uses the reading
 *   sigma = 2 pi int P b db of Eq. (18): pi bmax^2 P for area sampling; NaN
 *   for fixed-b instances (combine those with a b grid). */
#define QCAMS_XS_STRIDE 32
/* Per-group results of fixed impact-parameter grids, rows of
 * QCAMS_GRID_STRIDE doubles: [0] E_c (K), [1] v, [2] j, [3] number of b
 * values, [4] largest b, [5] trajectories, [6..9] sigma_x, [10..13] its
 * error, [14..17] rate k_x, for x = q, r1, r2, d; the rest 0. */
#define QCAMS_GRID_STRIDE 24
/* Gaussian-binning histograms, [n_inst][3][QCAMS_VMAX]: channel q, r1, r2 by
 * v_t, sum of w * W (Eq. (14) numerators). */
#define QCAMS_VMAX 64

typedef struct qcams_ctx qcams_ctx;

/* The system in its canonical form (Sec. 3.1 units, Sec. 3.2 pairs): masses
 * converted to electron masses (mass_unit = QCAMS_MASS_ME on return) and the
 * input forms QCAMS_MORSE_WE / QCAMS_LJ_EPS converted to QCAMS_MORSE /
 * QCAMS_LJ as documented above; other pairs copied.  qcams_create applies
 * the same conversion.  in, out: host (may alias).  Needs no device.
 * Errors (message from qcams_last_error(NULL)): EINVAL (unknown unit or
 * kind, non-positive masses, invalid pair parameters). */
int qcams_system_resolve(const qcams_system *in, qcams_system *out);

/* Create a context on `device` for one system and parameter set (the system
 * resolved as by qcams_system_resolve).  Finds the pair shapes (Buckingham
 * inner maximum, potential minimum, the maximum of r^3 V') on the device.
 * sync.  Errors: EINVAL (bad masses, units, kinds, LJ exponents, tolerances,
 * a potential without the single-well shape), EHIP, ENOMEM. */
int qcams_create(qcams_ctx **ctx, int device, const qcams_system *sys,
                 const qcams_params *prm);

/* Release the context and its device memory.  NULL is allowed. */
void qcams_destroy(qcams_ctx *ctx);

/* Message of the last error on this context (or of the last failed create
 * when ctx is NULL).  Owned by the library. */
const char *qcams_last_error(const qcams_ctx *ctx);

/* Bohr-Sommerfeld levels of AB (Eq. (10) with v' = v, Eq. (7)): for each of
 * n (v, j) pairs, out[4 i + 0..3] = E_vj (hartree), r-, r+ (turning points,
 * a0), tau_vj (vibrational period).  v, j, out: host.  sync.  Errors:
 * EUNBOUND (some level is not bound; its row is NaN), EINVAL. */
int qcams_levels(qcams_ctx *ctx, int32_t n, const int32_t *v, const int32_t *j, double *out);

/* Levels of AB from the Colbert-Miller DVR, the paper's internal-energy
 * method (Sec. 2.1; input keys npts, xmin, xmax of Sec. 3.1): E_vj is the
 * (v+1)-th lowest eigenvalue of the radial Hamiltonian with the centrifugal
 * term j(j+1)/(2 mu r^2) on the npts interior points of the box
 * (xmin, xmax) (particle-in-a-box form; one dense eigenproblem per distinct
 * j, reduced to tridiagonal form and bisected on the device); r-, r+ and
 * tau at that energy as in qcams_levels.  out: host [n][4].  sync.
 * Errors: EINVAL (grid: 16 <= npts <= 4096, 0 < xmin < xmax), EUNBOUND
 * (E_vj above the well), ENOROOT, ENOMEM, EHIP. */
int qcams_dvr_levels(qcams_ctx *ctx, int32_t npts, double xmin, double xmax, int32_t n,
                     const int32_t *v, const int32_t *j, double *out);

#define QCAMS_LEVELS_BS 0
#define QCAMS_LEVELS_DVR 1
/* Level method used by qcams_set_instances: QCAMS_LEVELS_BS (default,
 * Bohr-Sommerfeld, qcams_levels) or QCAMS_LEVELS_DVR with its grid
 * (qcams_dvr_levels).  host only.  Errors: EINVAL. */
int qcams_set_level_method(qcams_ctx *ctx, int32_t method, int32_t npts, double xmin, double xmax);

/* Install the instance table (host array of n_inst rows, sorted by
 * first_id, id ranges disjoint) and compute each instance's level on the
 * device with the context's level method.  sync.  Errors: EINVAL, EUNBOUND. */
int qcams_set_instances(qcams_ctx *ctx, const qcams_instance *inst, int32_t n_inst);

/* Initial conditions (Sec. 2.1, Eq. (5)-(6)) of trajectories ids[0..n)
 * (device int64, any order; each id must lie in an installed instance).
 * Writes st (all fields; h = 0, t = 0, status RUNNING, counters 0) and
 * sample [QCAMS_NS][st->ld] (device; may be NULL; its last row is the
 * importance weight, 1 except for QCAMS_B_PROPOSAL instances).  A trajectory
 * whose id is outside every instance, or whose b >= R, gets status
 * FAIL_NONFINITE.  async. */
int qcams_init_conditions(qcams_ctx *ctx, const int64_t *ids, int64_t n,
                          const qcams_state *st, double *sample, void *stream);

/* Integrate trajectories 0..n-1 of st with the adaptive RK integrator of
 * the context's variant (Eq. (3)-(4)) until each stops (status != RUNNING),
 * one lane per trajectory.  Trajectories already stopped are left
 * untouched.  async. */
int qcams_propagate(qcams_ctx *ctx, const qcams_state *st, int64_t n, void *stream);

/* qcams_propagate with a record of each trajectory's pair distances (the
 * quantities of the paper's trajectory plots, Sec. 2.2): the same steps as
 * qcams_propagate, and (t, r_AB, r_BC, r_CA) at the start and after every
 * accepted step written to rec (device [n][rec_max][4], trajectory-major),
 * the number of points written to rec_n (device int32 [n]; 0 for a
 * trajectory that was already stopped).  Past rec_max points a trajectory
 * continues unrecorded.  async.  Errors: EINVAL. */
int qcams_propagate_record(qcams_ctx *ctx, const qcams_state *st, int64_t n, double *rec,
                           int32_t rec_max, int32_t *rec_n, void *stream);

/* Product analysis (Sec. 2.2, Eq. (8)-(11)) of the final states 0..n-1.
 * async. */
int qcams_classify(qcams_ctx *ctx, const qcams_state *st, int64_t n, const qcams_outcome *out,
                   void *stream);

/* Per-instance opacities, Monte Carlo errors, cross sections, rates
 * (Eq. (12)-(16), (18)-(19)) and Gaussian-binning histograms (Eq. (14)-(15))
 * from n classified trajectories.  ids (device int64) must be sorted
 * ascending; weight (device, [n], may be NULL = all 1) are importance
 * weights.  xs: device [n_inst][QCAMS_XS_STRIDE]; hist: device
 * [n_inst][3][QCAMS_VMAX] or NULL.  async. */
int qcams_cross_sections(qcams_ctx *ctx, const qcams_outcome *out, const int64_t *ids,
                         const double *weight, int64_t n, double *xs, double *hist,
                         void *stream);

/* Fixed impact-parameter grids (the paper's Sec. 4 workflow): the installed
 * QCAMS_B_FIXED instances form groups of equal (E_c, v, j), each ordered by
 * b.  Number of groups, and (group_of, host [n_inst], may be NULL) the group
 * of every instance (-1 for other sampling modes).  host only.  Errors:
 * EINVAL. */
int qcams_grid_groups(qcams_ctx *ctx, int32_t *n_groups, int32_t *group_of);

/* Eq. (18)-(19) on every group: sigma_x = 2 pi int P_x(b) b db by the
 * trapezoid rule over the group's b values (reading: prefactor 2 pi, P a
 * probability; the integral runs from the smallest to the largest b), its
 * error from the independent per-b errors of xs, and the rate
 * k_x = sigma_x sqrt(2 E_c / mu_123).  xs: device [n_inst][QCAMS_XS_STRIDE]
 * as written by qcams_cross_sections or qcams_run; out: device
 * [n_groups][QCAMS_GRID_STRIDE].  No groups: nothing is written.  async.
 * Errors: EINVAL. */
int qcams_grid_cross_sections(qcams_ctx *ctx, const double *xs, double *out, void *stream);

/* Options of the fused persistent run. */
typedef struct {
    int32_t blocks;      /* persistent grid in 256-thread workgroups; 0 = 1 per compute unit */
    int32_t refill_min;  /* refill a wave once this many of its slots are idle (0 = 1) */
    int32_t check_every; /* trial steps between refill checks (0 = 1) */
    int32_t lpt;         /* 1: start instances longest-expected-first (cost ~ 1/(v_c sqrt(tau_vj))) */
    int32_t graph;       /* 1: capture the launch sequence once per buffer set and replay it */
    int32_t rk;          /* 0: the context's variant; 1: DOPRI5; 2: DOP853 */
    int32_t lanes;       /* lanes per trajectory: 1, 4 (a quad shares the arithmetic of one
                            trajectory; 16 slots per wave) or 8 (an octet; 8 slots per
                            wave).  All give bit-identical trajectories; 4 halves the
                            latency of a step, 8 takes about 5 % more off it, 1 has the
                            highest throughput.  0: 8 when every trajectory fits in the
                            grid's octet slots at once; else 4 when the expected step
                            count of the longest trajectory exceeds 2.1 x the total over
                            the lanes of a one-lane grid (a run bound by its longest
                            trajectories); else 1 */
    int32_t pad;
} qcams_run_opts;

/* The whole hot path over every installed trajectory (N = sum of n_traj):
 * initial conditions, propagation in one persistent launch whose slots (a
 * lane, a quad or an octet of lanes) take a new trajectory as soon as theirs stops,
 * classification, and the
 * per-instance reduction of qcams_cross_sections.  Results are stored at
 * each trajectory's natural position p (instances in id order, ids
 * consecutive inside an instance): st, sample (may be NULL), out, and
 * ids[p] (device int64 [N], written) as the matching trajectory id.  xs,
 * hist (may be NULL) as in qcams_cross_sections.  opts may be NULL
 * (defaults: 1 workgroup per CU, refill_min 1, check_every 8, LPT, no
 * graph, the context's RK variant, lanes chosen by run size).  The work
 * order (LPT or natural) is dealt to the 8 XCDs in chunks of 16 items and a
 * wave takes work from its own XCD's list before the others', so the state
 * lines a chunk touches stay in one L2.  Per-trajectory
 * results do not depend on blocks, refill_min, check_every, lpt, graph or
 * lanes.  With opts->graph the small set-up and analysis launches around
 * the persistent kernel are captured into two HIP graphs on first use (per
 * buffer set, order option and instance count) and replayed afterwards; the
 * persistent kernel is launched between them.  async.  Errors: EINVAL,
 * ENOMEM, EHIP. */
int qcams_run(qcams_ctx *ctx, const qcams_run_opts *opts, const qcams_state *st, double *sample,
              const qcams_outcome *out, int64_t *ids, double *xs, double *hist, void *stream);

/* qcams_run for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same per-trajectory and per-instance results as
 * qcams_run with graph = 0, but the run's work buffers (work-list counters,
 * work order, the reduction's per-chunk partial sums) live in a static
 * device array of 30,408,960 bytes that every GPU the library runs on holds
 * until the process ends; the call itself makes no hipMalloc, hipFree or
 * other allocating call.  Limits: at most 2,097,152 installed trajectories
 * and 8,192 reduction chunks (one per started 4096 trajectories of each
 * instance).  Every call on a GPU shares that GPU's array and leaves the
 * last run's contents in it (the counters are cleared by a kernel at the
 * start of each run): calls that overlap on one GPU -- on different streams
 * or from different contexts -- race and must be serialised by the caller.
 * The installed instance tables (qcams_set_instances) and the caller's
 * buffers are as for qcams_run; opts->graph must be 0.
 * qcams_last_run_kernel_ms, _wave_steps and _options report this run as
 * they do for qcams_run (the wave-step count until the next run on the
 * device overwrites the array).  async.  Errors: EINVAL (also beyond the
 * limits or with graph set), EHIP. */
int qcams_run_noalloc(qcams_ctx *ctx, const qcams_run_opts *opts, const qcams_state *st,
                      double *sample, const qcams_outcome *out, int64_t *ids, double *xs,
                      double *hist, void *stream);

/* Duration in milliseconds of the persistent propagation kernel of the last
 * qcams_run on this context, from HIP events recorded around that launch on
 * the run's stream (also when the run was a graph replay).  Waits for the
 * run to finish.  sync.  Errors: EINVAL (no run yet), EHIP. */
int qcams_last_run_kernel_ms(qcams_ctx *ctx, double *ms);

/* Iterations of the trial-step loop that the persistent waves of the last
 * qcams_run executed with at least one slot stepping (each such iteration
 * steps every running slot of its wave once).  Divided into the run's trial
 * steps (sum of nstep + nrej) it gives the slot utilisation, with
 * 64 / lanes slots per wave.  Waits for the run.  sync.  Errors: EINVAL (no
 * run yet), EHIP. */
int qcams_last_run_wave_steps(qcams_ctx *ctx, int64_t *wave_steps);

/* The options the last qcams_run on this context took effect with: blocks,
 * refill_min and check_every as clamped, rk = 1 (DOPRI5) or 2 (DOP853),
 * lanes = 1, 4 or 8.  host only.  Errors: EINVAL (no run yet). */
int qcams_last_run_options(qcams_ctx *ctx, qcams_run_opts *used);

/* Choose fast qcams_run options on the installed instances -- install a
 * calibration subset first -- by timing runs: coordinate descent, two
 * sweeps from the defaults, over lanes per trajectory (4, 1, 8), grid (1-4
 * workgroups per CU), refill_min (1, 4, 16), check_every (1, 4, 8) and
 * instance order (LPT, natural).  Returns the fastest in *best (graph off)
 * with its time in *best_ms (may be NULL).  Buffers as for qcams_run; each
 * option is run `reps` times and the minimum kept.  With search_rk = 1 the
 * RK variant is chosen first: DOPRI5 and DOP853 are each run with the
 * default schedule and the faster of those whose largest |H(t_f) - H(0)| /
 * escale over non-failed trajectories is below energy_gate (<= 0: no gate)
 * is kept (best->rk = 1 or 2); the variant changes per-trajectory results,
 * the schedule does not.  With search_rk = 0 the context's variant is used
 * (best->rk = 0).  Results are cached for the process, keyed by device,
 * search_rk / energy_gate, the number of installed trajectories and
 * instances, and a hash of the system, every integration parameter and the
 * installed instance table (so a workload of the same size but other
 * content is tuned afresh): with reps >= 0 a cached
 * result is returned without timing (reps = 0 counts as 1 otherwise); with
 * reps < 0 the search runs with |reps| repetitions and replaces the cached
 * result.  sync.  Errors as qcams_run; EINVAL also when no variant keeps
 * the gate. */
int qcams_autotune(qcams_ctx *ctx, const qcams_state *st, const qcams_outcome *out, int64_t *ids,
                   double *xs, int32_t reps, int32_t search_rk, double energy_gate,
                   qcams_run_opts *best, double *best_ms);

/* ======================================================================
 * Learned importance-sampling proposal.
 *
 * A network 6 -> 128 -> 128 -> 128 -> 4 (ReLU, softmax) estimates the
 * probabilities of the outcome classes (quench, r1, r2, dissociation) of a
 * trajectory from x = ((log10(E_c / K) - 3) / 2, b / 10 a0, v / 10, j / 10,
 * chi, cos theta).  Its forward and backward passes run on BF16 matrix cores
 * with FP32 accumulation; master weights, gradients and Adam state are FP32.
 * Flat parameter layout (float): W1[6][128], b1[128], W2[128][128], b2,
 * W3[128][128], b3, W4[128][4], b4 (W[i][o] input-major).
 * ====================================================================== */
#define QCAMS_MLP_NPARAM 34436
#define QCAMS_MLP_NIN 6
#define QCAMS_MLP_NOUT 4
/* proposal cells: 32 (b^2) x 16 (chi) x 16 (cos theta), index (ib*16 + ichi)*16 + icos */
#define QCAMS_PROP_CELLS 8192

typedef struct qcams_mlp qcams_mlp;

/* Create a network on `device`: params (host, [QCAMS_MLP_NPARAM]) or NULL
 * for He-uniform weights (U(+-sqrt(6/fan_in)) from a hash of (seed, index))
 * and zero biases.  Adam state zero.  sync.  Errors: ENOMEM, EHIP. */
int qcams_mlp_create(qcams_mlp **mlp, int device, const float *params, uint64_t seed);

/* Release the network.  NULL is allowed. */
void qcams_mlp_destroy(qcams_mlp *mlp);

/* Message of the last error on this network (or of the last failed create). */
const char *qcams_mlp_last_error(const qcams_mlp *mlp);

/* Copy the FP32 parameters to host memory [QCAMS_MLP_NPARAM].  sync. */
int qcams_mlp_get_params(qcams_mlp *mlp, float *params);

/* Replace the parameters (host [QCAMS_MLP_NPARAM]) and reset Adam.  sync. */
int qcams_mlp_set_params(qcams_mlp *mlp, const float *params);

/* Class probabilities prob (device [n][4] float) of inputs x (device [n][6]
 * float).  async. */
int qcams_mlp_forward(qcams_mlp *mlp, const float *x, int64_t n, float *prob, void *stream);

/* Gradient (device [QCAMS_MLP_NPARAM] float) of the mean softmax
 * cross-entropy over n rows: row r is x[idx[r]], y[idx[r]] (idx device int32
 * [n], or NULL for r itself); labels y (device int32) in 0..3, a negative
 * label contributes nothing (the mean still divides by n).  loss (device
 * [1] float, may be NULL) receives the mean loss.  async. */
int qcams_mlp_gradient(qcams_mlp *mlp, const float *x, const int32_t *y, const int32_t *idx,
                       int64_t n, float *grad, float *loss, void *stream);

/* One Adam step (Kingma & Ba 2015; beta 0.9 / 0.999, eps 1e-8) with the
 * gradient grad (device [QCAMS_MLP_NPARAM]).  async. */
int qcams_mlp_adam(qcams_mlp *mlp, const float *grad, float lr, void *stream);

/* One epoch of minibatch training: batches of `batch` rows taken in the
 * order perm (device int32 [n]; full batches only), each a gradient and an
 * Adam step.  loss_sum (device [1] float) receives the sum of the batch
 * losses.  The epoch's launches are captured once per argument set and
 * replayed (update perm between epochs).  async. */
int qcams_mlp_train_epoch(qcams_mlp *mlp, const float *x, const int32_t *y, const int32_t *perm,
                          int64_t n, int32_t batch, float lr, float *loss_sum, void *stream);

/* Network inputs and labels of classified trajectories: x (device [n][6]
 * float) from each trajectory's instance (ids, device int64 [n]) and sample
 * (device [QCAMS_NS][sample_ld]); y (device int32 [n]) = the label for
 * quench / r1 / r2 / dissociation, -1 otherwise.  async. */
int qcams_mlp_features(qcams_ctx *ctx, const int64_t *ids, const double *sample, int64_t sample_ld,
                       const qcams_outcome *out, int64_t n, float *x, int32_t *y, void *stream);

/* Build and install the proposal used by instances with b_mode
 * QCAMS_B_PROPOSAL: for installed instance `inst` the network's probability
 * pi_k of class `channel` at the centre of each cell k gives
 * q_k = alpha / K + (1 - alpha) sqrt(pi_k) / sum_l sqrt(pi_l)  (K cells;
 * alpha in (0, 1] keeps every weight <= 1/alpha).  A trajectory picks cell k
 * with probability q_k and a uniform point inside it, and carries the weight
 * (1/K) / q_k (1 exactly when alpha = 1).  q (device [QCAMS_PROP_CELLS]
 * double, may be NULL) receives the table.  mlp may be NULL only with
 * alpha = 1.  sync.  Errors: EINVAL, EHIP. */
int qcams_proposal_build(qcams_ctx *ctx, qcams_mlp *mlp, int32_t inst, int32_t channel,
                         double alpha, double *q);

/* Install a given proposal table (host [QCAMS_PROP_CELLS], every entry > 0;
 * normalised by the library) for QCAMS_B_PROPOSAL instances.  sync.
 * Errors: EINVAL, ENOMEM, EHIP. */
int qcams_proposal_set(qcams_ctx *ctx, const double *q);

#ifdef __cplusplus
}
#endif

#endif /* QCAMS_H */
