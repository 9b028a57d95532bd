// qcams_api.hip -- kernels and C-ABI entry points of the QCT library (gfx950).
//
// One trajectory per lane, state in structure-of-arrays HBM buffers, all
// arithmetic FP64.  See include/qcams.h for the contract of each call.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/qcams.h"
#include "qcams_device.h"

using namespace qd;

struct qcams_ctx {
    int device = 0;
    Sys sys{};
    Prm prm{};
    int kinds = 0;               // kind triple packed as k0 + 3 k1 + 9 k2
    Inst* d_inst = nullptr;      // device instance table
    int32_t n_inst = 0;
    std::vector<Inst> h_inst;
    char err[512] = {0};
};

static char g_create_err[512];

static int fail(qcams_ctx* c, int code, const char* fmt, ...)
{
    char* dst = c ? c->err : g_create_err;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(dst, 512, fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_OK(ctx, expr)                                                              \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(ctx, QCAMS_EHIP, "%s: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

// ---------------------------------------------------------------------------
// set-up kernels
// ---------------------------------------------------------------------------
__global__ void k_shapes(Pot p0, Pot p1, Pot p2, Shape* out, int* rc)
{
    const int i = threadIdx.x;
    if (i >= 3) return;
    const Pot P = i == 0 ? p0 : (i == 1 ? p1 : p2);
    Shape s{};
    rc[i] = pair_shape(P, s);
    out[i] = s;
}

__global__ void k_levels(Pot P, Shape Sh, double mu, int n, const int* v, const int* j,
                         double* out, int* rc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double o[4] = {NAN, NAN, NAN, NAN};
    rc[i] = bs_level(P, Sh, mu, v[i], j[i], o);
    if (rc[i] != 0) o[0] = o[1] = o[2] = o[3] = NAN;
    for (int k = 0; k < 4; ++k) out[4 * i + k] = o[k];
}

// ---------------------------------------------------------------------------
// initial conditions
// ---------------------------------------------------------------------------
__device__ inline int find_instance(const Inst* inst, int n_inst, int64_t id)
{
    int lo = 0, hi = n_inst - 1, k = -1;
    while (lo <= hi) {   // last instance with first_id <= id
        const int mid = (lo + hi) >> 1;
        if (inst[mid].first_id <= id) { k = mid; lo = mid + 1; }
        else hi = mid - 1;
    }
    if (k < 0 || id >= inst[k].first_id + inst[k].n_traj) return -1;
    return k;
}

__global__ void k_init(Sys S, Prm P, const Inst* inst, int n_inst, const int64_t* ids,
                       int64_t n, double* d, int32_t* nstep, int32_t* nrej, uint8_t* status,
                       int64_t ld, double* sample)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t id = ids[i];
    const int k = find_instance(inst, n_inst, id);
    double x[6] = {0, 0, 0, 0, 0, 0}, p[6] = {0, 0, 0, 0, 0, 0}, smp[5] = {0, 0, 0, 0, 0};
    double tmax = 0.0, rstop = 0.0, e0 = 0.0, esc = 1.0;
    uint8_t st = RUNNING;
    if (k < 0) {
        st = FAIL_NONFINITE;
    } else {
        const Inst I = inst[k];
        if (!initial_state(S, P, I, id, x, p, tmax, rstop, smp)) st = FAIL_NONFINITE;
        e0 = hamiltonian(S, x, p);
        esc = fmax(fabs(e0), fabs(I.Evj));
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        d[f * ld + i] = x[f];
        d[(6 + f) * ld + i] = p[f];
    }
    d[QCAMS_F_T * ld + i] = 0.0;
    d[QCAMS_F_TMAX * ld + i] = tmax;
    d[QCAMS_F_RSTOP * ld + i] = rstop;
    d[QCAMS_F_E0 * ld + i] = e0;
    d[QCAMS_F_ESCALE * ld + i] = esc;
    d[QCAMS_F_H * ld + i] = 0.0;
    nstep[i] = 0;
    nrej[i] = 0;
    status[i] = st;
    if (sample) {
        for (int f = 0; f < 5; ++f) sample[f * ld + i] = smp[f];
        sample[5 * ld + i] = 1.0;
    }
}

// ---------------------------------------------------------------------------
// propagation: one trajectory per lane until it stops
// ---------------------------------------------------------------------------
template <int K0, int K1, int K2>
__global__ void __launch_bounds__(256) k_propagate(Sys S, Prm P, double* d, int32_t* nstep,
                                                   int32_t* nrej, uint8_t* status, int64_t ld,
                                                   int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (status[i] != RUNNING) return;
    Lane L;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        L.x[f] = d[f * ld + i];
        L.p[f] = d[(6 + f) * ld + i];
    }
    L.t = d[QCAMS_F_T * ld + i];
    L.tmax = d[QCAMS_F_TMAX * ld + i];
    const double rs = d[QCAMS_F_RSTOP * ld + i];
    L.rstop2 = rs * rs;
    L.h = d[QCAMS_F_H * ld + i];
    L.nstep = nstep[i];
    L.nrej = nrej[i];
    L.status = RUNNING;
    L.last_rej = 0;
    double s2[3];
    force<K0, K1, K2>(S, L.x, L.F, s2);
    if (P.fixed_step) L.h = P.h_fixed;
    else if (!(L.h > 0.0))
        L.h = initial_step<K0, K1, K2>(S, L.x, L.p, L.F, P.atol, P.rtol, L.tmax - L.t);
    if (!is_finite(L.t) || !is_finite(L.tmax) || !is_finite(L.h)) L.status = FAIL_NONFINITE;
    else if (L.t >= L.tmax) L.status = OK_TMAX;
    else if (L.nstep >= P.max_steps) L.status = FAIL_MAXSTEPS;
    while (L.status == RUNNING) lane_step<K0, K1, K2>(S, P, L);
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        d[f * ld + i] = L.x[f];
        d[(6 + f) * ld + i] = L.p[f];
    }
    d[QCAMS_F_T * ld + i] = L.t;
    d[QCAMS_F_H * ld + i] = L.h;
    nstep[i] = L.nstep;
    nrej[i] = L.nrej;
    status[i] = (uint8_t)L.status;
}

// ---------------------------------------------------------------------------
// classification
// ---------------------------------------------------------------------------
__global__ void k_classify(Sys S, Prm P, const double* d, const uint8_t* status, int64_t ld,
                           int64_t n, uint8_t* label, int16_t* vt, int16_t* jt, double* od,
                           int64_t old)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x[6], p[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        x[f] = d[f * ld + i];
        p[f] = d[(6 + f) * ld + i];
    }
    const int st = status[i];
    Outcome o;
    o.label = FAILED;
    o.vt = o.jt = 0;
    o.vprime = o.jprime = o.w = 0.0;
    if (st == OK_RSTOP || st == OK_TMAX) o = classify_state(S, P, x, p);
    const double dE = (hamiltonian(S, x, p) - d[QCAMS_F_E0 * ld + i]) / d[QCAMS_F_ESCALE * ld + i];
    label[i] = (uint8_t)o.label;
    vt[i] = (int16_t)o.vt;
    jt[i] = (int16_t)o.jt;
    od[0 * old + i] = o.vprime;
    od[1 * old + i] = o.jprime;
    od[2 * old + i] = o.w;
    od[3 * old + i] = dE;
}

// ---------------------------------------------------------------------------
// per-instance reduction: one 256-thread block per instance, fixed order
// ---------------------------------------------------------------------------
constexpr int kRedThreads = 256;

__device__ inline int64_t lower_bound_ids(const int64_t* ids, int64_t n, int64_t key)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (ids[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// tree reduction of NV doubles per thread over the block; result in red[0..NV)
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double* red)
{
    const int t = threadIdx.x;
    for (int k = 0; k < NV; ++k) red[k * kRedThreads + t] = v[k];
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (t < s)
            for (int k = 0; k < NV; ++k) red[k * kRedThreads + t] += red[k * kRedThreads + t + s];
        __syncthreads();
    }
    for (int k = 0; k < NV; ++k) v[k] = red[k * kRedThreads];
    __syncthreads();
}

__global__ void __launch_bounds__(kRedThreads)
k_xsec(const Inst* inst, int n_inst, double mu123, const uint8_t* label, const int16_t* vt,
       const double* od, int64_t old, const int64_t* ids, const double* weight, int64_t n,
       double* xs, double* hist)
{
    const int k = blockIdx.x;
    if (k >= n_inst) return;
    __shared__ double red[16 * kRedThreads];
    const Inst I = inst[k];
    const int64_t b = lower_bound_ids(ids, n, I.first_id);
    const int64_t e = lower_bound_ids(ids, n, I.first_id + I.n_traj);
    // 0..5 counts, 6..9 sum w 1[x], 10..13 sum (w 1[x])^2, 14 sum w, 15 sum w^2
    double acc[16];
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    double vtmax = -1.0;
    for (int64_t i = b + threadIdx.x; i < e; i += kRedThreads) {
        const int c = label[i];
        const double w = weight ? weight[i] : 1.0;
        if (c < 6) acc[c] += 1.0;
        if (c < 4) {
            acc[6 + c] += w;
            acc[10 + c] += w * w;
        }
        acc[14] += w;
        acc[15] += w * w;
        if (c < 3) vtmax = fmax(vtmax, (double)vt[i]);
    }
    block_sum<16>(acc, red);
    double m1[1] = {vtmax};
    // max-reduce through the same buffer
    red[threadIdx.x] = m1[0];
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const int vmax_here = (int)fmin(red[0], (double)(QCAMS_VMAX - 1));
    __syncthreads();
    // Gaussian-binning histogram, one fixed-order reduction per (channel, vt)
    double Wsum = 0.0;
    for (int c = 0; c < 3; ++c) {
        for (int v = 0; v <= vmax_here; ++v) {
            double h[1] = {0.0};
            for (int64_t i = b + threadIdx.x; i < e; i += kRedThreads) {
                if (label[i] == c && vt[i] == v) {
                    const double w = weight ? weight[i] : 1.0;
                    h[0] += w * od[2 * old + i];
                }
            }
            block_sum<1>(h, red);
            Wsum += h[0];
            if (hist && threadIdx.x == 0) hist[((int64_t)k * 3 + c) * QCAMS_VMAX + v] = h[0];
        }
        if (hist && threadIdx.x == 0)
            for (int v = vmax_here + 1; v < QCAMS_VMAX; ++v)
                hist[((int64_t)k * 3 + c) * QCAMS_VMAX + v] = 0.0;
    }
    if (threadIdx.x != 0) return;
    double* row = xs + (int64_t)k * QCAMS_XS_STRIDE;
    const double N = (double)(e - b);
    row[0] = N;
    for (int c = 0; c < 6; ++c) row[1 + c] = acc[c];
    const double area = I.b_mode == QCAMS_B_AREA ? kPi * I.bmax * I.bmax : NAN;
    const double speed = sqrt(2.0 * I.Ec / mu123);
    for (int c = 0; c < 4; ++c) {
        const double m = N > 0 ? acc[6 + c] / N : NAN;
        const double var = N > 0 ? acc[10 + c] / N - m * m : NAN;
        const double se = sqrt(fmax(var, 0.0) / N);
        row[7 + c] = m;
        row[11 + c] = se;
        row[15 + c] = area * m;
        row[19 + c] = area * se;
        row[23 + c] = area * m * speed;
    }
    // Eq. (15): W = sum over bins of the weights of q and r products, plus N_d
    row[27] = Wsum + acc[6 + DISS];
    row[28] = acc[14];
    row[29] = acc[15];
    row[30] = 0.0;
    row[31] = 0.0;
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
static int grid_of(int64_t n, int threads) { return (int)((n + threads - 1) / threads); }

static bool pair_ok(const qcams_pair& p)
{
    if (p.kind == QCAMS_MORSE) return p.p[0] >= 0.0 && p.p[2] > 0.0;
    if (p.kind == QCAMS_LJ) return p.n > p.m && p.m >= 3 && p.n <= 64 && p.p[0] > 0 && p.p[1] > 0;
    if (p.kind == QCAMS_BUCK) return p.p[0] > 0.0 && p.p[1] > 0.0 && p.p[2] > 0.0;
    return false;
}

static bool pot_is_zero(const qcams_pair& p) { return p.kind == QCAMS_MORSE && p.p[0] == 0.0; }

template <int K0, int K1, int K2>
static void launch_propagate(qcams_ctx* c, const qcams_state* st, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL((k_propagate<K0, K1, K2>), dim3(grid_of(n, 256)), dim3(256), 0, s, c->sys,
                       c->prm, st->d, st->nstep, st->nrej, st->status, st->ld, n);
}

extern "C" {

int qcams_create(qcams_ctx** out, int device, const qcams_system* sys, const qcams_params* prm)
{
    if (!out || !sys || !prm) return fail(nullptr, QCAMS_EINVAL, "null argument");
    *out = nullptr;
    for (int i = 0; i < 3; ++i)
        if (!(sys->mass[i] > 0.0)) return fail(nullptr, QCAMS_EINVAL, "mass %d must be > 0", i);
    for (int i = 0; i < 3; ++i)
        if (!pair_ok(sys->pair[i]))
            return fail(nullptr, QCAMS_EINVAL, "pair %d: unsupported kind or parameters", i);
    if (!(prm->atol > 0.0) || !(prm->rtol >= 0.0) || !(prm->t_stop > 0.0) || !(prm->r_stop > 0.0) ||
        !(prm->R0 > 0.0) || !(prm->gb_sigma > 0.0) || prm->max_steps < 1 ||
        prm->max_steps > 2147483647LL || (prm->fixed_step && !(prm->h_fixed > 0.0)))
        return fail(nullptr, QCAMS_EINVAL, "invalid integration parameters");
    qcams_ctx* c = new (std::nothrow) qcams_ctx();
    if (!c) return fail(nullptr, QCAMS_ENOMEM, "host allocation failed");
    c->device = device;
    int rc = QCAMS_OK;
    {
        hipError_t e = hipSetDevice(device);
        if (e != hipSuccess) {
            delete c;
            return fail(nullptr, QCAMS_EHIP, "hipSetDevice(%d): %s", device, hipGetErrorString(e));
        }
    }
    const double mA = sys->mass[0], mB = sys->mass[1], mC = sys->mass[2];
    Sys& S = c->sys;
    for (int i = 0; i < 3; ++i) {
        const qcams_pair& q = sys->pair[i];
        S.pot[i].kind = q.kind;
        S.pot[i].n = q.n;
        S.pot[i].m = q.m;
        S.pot[i].p0 = q.p[0];
        S.pot[i].p1 = q.p[1];
        S.pot[i].p2 = q.p[2];
    }
    // reduced masses, Eq. (2)
    S.mu12 = 1.0 / (1.0 / mA + 1.0 / mB);
    S.mu123 = 1.0 / (1.0 / mC + 1.0 / (mA + mB));
    S.inv_mu12 = 1.0 / S.mu12;
    S.inv_mu123 = 1.0 / S.mu123;
    S.mu_pair[0] = S.mu12;
    S.mu_pair[1] = 1.0 / (1.0 / mB + 1.0 / mC);
    S.mu_pair[2] = 1.0 / (1.0 / mC + 1.0 / mA);
    S.cA = mA / (mA + mB);
    S.cB = mB / (mA + mB);
    // pair shapes on the device (a switched-off Morse pair has none)
    Shape* d_sh = nullptr;
    int* d_rc = nullptr;
    Shape h_sh[3];
    int h_rc[3];
    if (hipMalloc(&d_sh, 3 * sizeof(Shape)) != hipSuccess ||
        hipMalloc(&d_rc, 3 * sizeof(int)) != hipSuccess) {
        (void)hipFree(d_sh);
        delete c;
        return fail(nullptr, QCAMS_ENOMEM, "device allocation failed");
    }
    hipLaunchKernelGGL(k_shapes, dim3(1), dim3(64), 0, 0, S.pot[0], S.pot[1], S.pot[2], d_sh,
                       d_rc);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(h_sh, d_sh, sizeof h_sh, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(h_rc, d_rc, sizeof h_rc, hipMemcpyDeviceToHost);
    (void)hipFree(d_sh);
    (void)hipFree(d_rc);
    if (e != hipSuccess) {
        delete c;
        return fail(nullptr, QCAMS_EHIP, "pair shapes: %s", hipGetErrorString(e));
    }
    for (int i = 0; i < 3; ++i) {
        if (pot_is_zero(sys->pair[i])) {
            h_sh[i] = Shape{0.0, sys->pair[i].p[1], 2.0 * sys->pair[i].p[1], 0.0};
            continue;
        }
        if (h_rc[i] != 0) {
            delete c;
            return fail(nullptr, QCAMS_EINVAL,
                        "pair %d: potential has no single well / barrier structure", i);
        }
    }
    for (int i = 0; i < 3; ++i) {
        S.shape[i] = h_sh[i];
        S.rin2[i] = h_sh[i].rin * h_sh[i].rin;
    }
    int kk[3];
    for (int i = 0; i < 3; ++i) kk[i] = sys->pair[i].kind;
    c->kinds = kk[0] + 3 * kk[1] + 9 * kk[2];
    c->prm.R0 = prm->R0;
    c->prm.t_stop = prm->t_stop;
    c->prm.r_stop = prm->r_stop;
    c->prm.atol = prm->atol;
    c->prm.rtol = prm->rtol;
    c->prm.gb_sigma = prm->gb_sigma;
    c->prm.h_fixed = prm->h_fixed;
    c->prm.fixed_step = prm->fixed_step;
    c->prm.literal_bound = prm->literal_bound;
    c->prm.max_steps = prm->max_steps;
    *out = c;
    return rc;
}

void qcams_destroy(qcams_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->d_inst) (void)hipFree(c->d_inst);
    delete c;
}

const char* qcams_last_error(const qcams_ctx* c) { return c ? c->err : g_create_err; }

int qcams_levels(qcams_ctx* c, int32_t n, const int32_t* v, const int32_t* j, double* out)
{
    if (!c) return fail(nullptr, QCAMS_EINVAL, "null context");
    if (n < 0 || (n > 0 && (!v || !j || !out))) return fail(c, QCAMS_EINVAL, "bad arguments");
    if (n == 0) return QCAMS_OK;
    for (int i = 0; i < n; ++i)
        if (v[i] < 0 || j[i] < 0) return fail(c, QCAMS_EINVAL, "negative quantum number");
    HIP_OK(c, hipSetDevice(c->device));
    int *dv = nullptr, *dj = nullptr, *drc = nullptr;
    double* dout = nullptr;
    std::vector<int> rc(n);
    hipError_t e = hipMalloc(&dv, n * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&dj, n * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&drc, n * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&dout, 4 * (size_t)n * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(dv, v, n * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dj, j, n * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_levels, dim3(grid_of(n, 64)), dim3(64), 0, 0, c->sys.pot[0],
                           c->sys.shape[0], c->sys.mu12, n, dv, dj, dout, drc);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(out, dout, 4 * (size_t)n * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(rc.data(), drc, n * sizeof(int), hipMemcpyDeviceToHost);
    (void)hipFree(dv);
    (void)hipFree(dj);
    (void)hipFree(drc);
    (void)hipFree(dout);
    if (e != hipSuccess) return fail(c, QCAMS_EHIP, "levels: %s", hipGetErrorString(e));
    for (int i = 0; i < n; ++i) {
        if (rc[i] == -2) return fail(c, QCAMS_EUNBOUND, "level v=%d j=%d is not bound", v[i], j[i]);
        if (rc[i] != 0) return fail(c, QCAMS_ENOROOT, "level v=%d j=%d: no root", v[i], j[i]);
    }
    return QCAMS_OK;
}

int qcams_set_instances(qcams_ctx* c, const qcams_instance* inst, int32_t n_inst)
{
    if (!c) return fail(nullptr, QCAMS_EINVAL, "null context");
    if (n_inst < 1 || !inst) return fail(c, QCAMS_EINVAL, "need at least one instance");
    std::vector<Inst> h(n_inst);
    std::vector<int32_t> vv(n_inst), jj(n_inst);
    for (int k = 0; k < n_inst; ++k) {
        const qcams_instance& q = inst[k];
        if (!(q.Ec_K > 0.0) || q.n_traj < 0 || q.first_id < 0 ||
            (q.b_mode != QCAMS_B_FIXED && q.b_mode != QCAMS_B_AREA) ||
            (q.b_mode == QCAMS_B_FIXED && !(q.b >= 0.0)) ||
            (q.b_mode == QCAMS_B_AREA && !(q.bmax >= 0.0)))
            return fail(c, QCAMS_EINVAL, "instance %d: invalid fields", k);
        if (k > 0 && q.first_id < inst[k - 1].first_id + inst[k - 1].n_traj)
            return fail(c, QCAMS_EINVAL, "instance %d: ids overlap or are not sorted", k);
        // kelvin -> hartree (Boltzmann constant in E_h / K, CODATA 2018)
        h[k].Ec = q.Ec_K * 3.1668115634556e-6;
        h[k].b = q.b;
        h[k].bmax = q.bmax;
        h[k].b_mode = q.b_mode;
        h[k].v = q.v;
        h[k].j = q.j;
        h[k].n_traj = q.n_traj;
        h[k].first_id = q.first_id;
        h[k].seed = q.seed;
        vv[k] = q.v;
        jj[k] = q.j;
    }
    std::vector<double> lev(4 * (size_t)n_inst);
    int rc = qcams_levels(c, n_inst, vv.data(), jj.data(), lev.data());
    if (rc != QCAMS_OK) return rc;
    for (int k = 0; k < n_inst; ++k) {
        h[k].Evj = lev[4 * k + 0];
        h[k].rminus = lev[4 * k + 1];
        h[k].rplus = lev[4 * k + 2];
        h[k].tau = lev[4 * k + 3];
        const double b = inst[k].b_mode == QCAMS_B_AREA ? inst[k].bmax : inst[k].b;
        if (!(b < c->prm.R0)) return fail(c, QCAMS_EINVAL, "instance %d: impact parameter >= R0", k);
    }
    HIP_OK(c, hipSetDevice(c->device));
    if (c->d_inst) {
        HIP_OK(c, hipFree(c->d_inst));
        c->d_inst = nullptr;
    }
    if (hipMalloc(&c->d_inst, n_inst * sizeof(Inst)) != hipSuccess) {
        c->d_inst = nullptr;
        c->n_inst = 0;
        return fail(c, QCAMS_ENOMEM, "instance table allocation failed");
    }
    HIP_OK(c, hipMemcpy(c->d_inst, h.data(), n_inst * sizeof(Inst), hipMemcpyHostToDevice));
    c->n_inst = n_inst;
    c->h_inst = h;
    return QCAMS_OK;
}

static int check_state(qcams_ctx* c, const qcams_state* st, int64_t n)
{
    if (!st || n < 0) return fail(c, QCAMS_EINVAL, "bad state or size");
    if (n > 0 && (!st->d || !st->nstep || !st->nrej || !st->status || st->ld < n))
        return fail(c, QCAMS_EINVAL, "state buffers missing or ld < n");
    return QCAMS_OK;
}

int qcams_init_conditions(qcams_ctx* c, const int64_t* ids, int64_t n, const qcams_state* st,
                          double* sample, void* stream)
{
    if (!c) return fail(nullptr, QCAMS_EINVAL, "null context");
    if (int rc = check_state(c, st, n)) return rc;
    if (c->n_inst < 1) return fail(c, QCAMS_EINVAL, "no instances installed");
    if (n == 0) return QCAMS_OK;
    if (!ids) return fail(c, QCAMS_EINVAL, "null ids");
    HIP_OK(c, hipSetDevice(c->device));
    hipLaunchKernelGGL(k_init, dim3(grid_of(n, 256)), dim3(256), 0, (hipStream_t)stream, c->sys,
                       c->prm, c->d_inst, c->n_inst, ids, n, st->d, st->nstep, st->nrej,
                       st->status, st->ld, sample);
    HIP_OK(c, hipGetLastError());
    return QCAMS_OK;
}

int qcams_propagate(qcams_ctx* c, const qcams_state* st, int64_t n, void* stream)
{
    if (!c) return fail(nullptr, QCAMS_EINVAL, "null context");
    if (int rc = check_state(c, st, n)) return rc;
    if (n == 0) return QCAMS_OK;
    HIP_OK(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    if (c->kinds == 0) launch_propagate<0, 0, 0>(c, st, n, s);
    else if (c->kinds == QCAMS_LJ + 3 * QCAMS_MORSE + 9 * QCAMS_BUCK) launch_propagate<1, 0, 2>(c, st, n, s);
    else launch_propagate<-1, -1, -1>(c, st, n, s);
    HIP_OK(c, hipGetLastError());
    return QCAMS_OK;
}

int qcams_classify(qcams_ctx* c, const qcams_state* st, int64_t n, const qcams_outcome* out,
                   void* stream)
{
    if (!c) return fail(nullptr, QCAMS_EINVAL, "null context");
    if (int rc = check_state(c, st, n)) return rc;
    if (!out || (n > 0 && (!out->label || !out->vt || !out->jt || !out->d || out->ld < n)))
        return fail(c, QCAMS_EINVAL, "outcome buffers missing or ld < n");
    if (n == 0) return QCAMS_OK;
    HIP_OK(c, hipSetDevice(c->device));
    hipLaunchKernelGGL(k_classify, dim3(grid_of(n, 128)), dim3(128), 0, (hipStream_t)stream,
                       c->sys, c->prm, st->d, st->status, st->ld, n, out->label, out->vt, out->jt,
                       out->d, out->ld);
    HIP_OK(c, hipGetLastError());
    return QCAMS_OK;
}

int qcams_cross_sections(qcams_ctx* c, const qcams_outcome* out, const int64_t* ids,
                         const double* weight, int64_t n, double* xs, double* hist, void* stream)
{
    if (!c) return fail(nullptr, QCAMS_EINVAL, "null context");
    if (c->n_inst < 1) return fail(c, QCAMS_EINVAL, "no instances installed");
    if (!out || !xs || n < 0 || (n > 0 && (!ids || !out->label || !out->vt || !out->d || out->ld < n)))
        return fail(c, QCAMS_EINVAL, "bad arguments");
    HIP_OK(c, hipSetDevice(c->device));
    hipLaunchKernelGGL(k_xsec, dim3(c->n_inst), dim3(kRedThreads), 0, (hipStream_t)stream,
                       c->d_inst, c->n_inst, c->sys.mu123, out->label, out->vt, out->d, out->ld,
                       ids, weight, n, xs, hist);
    HIP_OK(c, hipGetLastError());
    return QCAMS_OK;
}

}  // extern "C"
