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
#include <algorithm>
#include <functional>
#include <map>
#include <mutex>
#include <tuple>
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
    int32_t inst_cap = 0;        // capacity of the device instance tables
    std::vector<Inst> h_inst;
    // fixed-b grids: instances grouped by (E_c, v, j), sorted by b
    int32_t* d_grid_inst = nullptr;   // [n_fixed] instance indices, group by group
    int32_t* d_grid_off = nullptr;    // [n_groups + 1]
    int32_t n_groups = 0, grid_cap = 0;
    std::vector<int32_t> h_group_of;  // [n_inst] group of each instance, -1 if none
    int64_t n_total = 0;          // sum of n_traj
    int32_t* d_id_inst = nullptr;    // [n_inst] identity order
    // longest-expected-first order of the instances for the persistent run
    int32_t* d_lpt_inst = nullptr;   // [n_inst] instance index by LPT rank
    int64_t* d_lpt_off = nullptr;    // [n_inst + 1] work offsets in LPT order
    int64_t* d_nat_off = nullptr;    // [n_inst + 1] natural (id-sorted) offsets
    unsigned long long* d_counter = nullptr;   // [kCounters] of the persistent run: work cursors, wave steps
    int64_t* d_order = nullptr;                // [n_total] work item -> natural position
    int64_t order_cap = 0;
    // per-instance reduction in chunks of positions: chunk offsets per
    // instance and one partial-sum row per chunk
    int64_t* d_xoff = nullptr;    // [n_inst + 1]
    double* d_xpart = nullptr;    // [n_xchunks][kPartStride]
    int64_t n_xchunks = 0, xoff_cap = 0, xpart_cap = 0;
    hipEvent_t ev_prop[2] = {nullptr, nullptr};   // around the persistent launch
    unsigned long long* last_counter = nullptr;   // counters of the last run (context or scratch)
    qcams_run_opts last_opts{};                   // effective options of the last run
    bool lj126 = false;                           // pair AB is LJ 12-6
    double cost_max = 0.0, cost_total = 0.0;      // expected steps: largest, summed
    int level_method = QCAMS_LEVELS_BS;           // levels of qcams_set_instances
    int dvr_npts = 0;
    double dvr_xmin = 0.0, dvr_xmax = 0.0;
    bool has_run = false;
    // importance-sampling proposal (cells of b^2, chi, cos theta)
    double* d_prop_q = nullptr;
    double* d_prop_cdf = nullptr;
    float* d_cell_x = nullptr;   // network inputs at the cell centres
    float* d_cell_p = nullptr;   // network outputs
    int n_cu = 0;
    // captured launch sequence of qcams_run
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr, graph2_exec = nullptr;
    hipGraph_t graph = nullptr, graph2 = nullptr;
    uint64_t graph_key[18] = {0};
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

// One wave per level: every lane runs the same root finding (the same
// values, so the control flow is uniform) and lane k < kNQ evaluates
// quadrature node k; the node sums are a butterfly over the wave, which
// leaves the same bits in every lane.
__global__ void __launch_bounds__(64) k_levels(Pot P, Shape Sh, double mu, int n, const int* v,
                                               const int* j, double* out, int* rc)
{
    const int i = blockIdx.x;
    if (i >= n) return;
    const int k = threadIdx.x;
    double st = 0.0, ct = 0.0;
    if (k < kNQ) sincos(kPi * (k + 0.5) / kNQ, &st, &ct);
    auto ap = [&](double J2, double E, double rm, double rp, double& act, double& per) {
        const double c = 0.5 * (rp + rm), h = 0.5 * (rp - rm);
        double a = 0.0, q = 0.0;
        if (k < kNQ) ap_node(P, J2 / (2.0 * mu), E, c, h, st, ct, a, q);
        for (int m = 32; m >= 1; m >>= 1) {
            a += __shfl_xor(a, m);
            q += __shfl_xor(q, m);
        }
        ap_finish(mu, h, a, q, act, per);
    };
    double o[4] = {NAN, NAN, NAN, NAN};
    const int r = bs_level_with(P, Sh, mu, v[i], j[i], o, ap);
    if (r != 0) o[0] = o[1] = o[2] = o[3] = NAN;
    if (k == 0) {
        rc[i] = r;
        for (int f = 0; f < 4; ++f) out[4 * i + f] = o[f];
    }
}

// turning points and period at given energies (the DVR levels)
__global__ void k_levels_at(Pot P, Shape Sh, double mu, int n, const double* E, const int* j,
                            double* out, int* rc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double o[4] = {NAN, NAN, NAN, NAN};
    rc[i] = level_at_energy(P, Sh, mu, j[i], E[i], o);
    if (rc[i] != 0) o[1] = o[2] = o[3] = NAN;
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

template <int K0, int K1, int K2, int RK>
__global__ void __launch_bounds__(256)
k_init(Sys S, Prm P, const Inst* inst, int n_inst, const int64_t* ids, int64_t n, double* d,
       int32_t* nstep, int32_t* nrej, uint8_t* status, int64_t ld, double* sample,
       const double* prop_q, const double* prop_cdf)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t id = ids[i];
    const int k = find_instance(inst, n_inst, id);
    double x[6] = {0, 0, 0, 0, 0, 0}, p[6] = {0, 0, 0, 0, 0, 0}, smp[6] = {0, 0, 0, 0, 0, 1};
    double tmax = 0.0, rstop = 0.0, e0 = 0.0, esc = 1.0, h = 0.0;
    uint8_t st = RUNNING;
    if (k < 0) {
        st = FAIL_NONFINITE;
    } else {
        const Inst I = inst[k];
        if (I.b_mode == 2 && !prop_q) st = FAIL_NONFINITE;
        else if (!initial_state(S, P, I, id, x, p, tmax, rstop, smp, prop_q, prop_cdf)) st = FAIL_NONFINITE;
        e0 = hamiltonian(S, x, p);
        esc = fmax(fabs(e0), fabs(I.Evj));
        // starting step of the RK5(4) controller (fixed step: h_fixed)
        if (st == RUNNING) {
            double F[6], s2[3];
            force<K0, K1, K2>(S, x, F, s2);
            h = P.fixed_step ? P.h_fixed : initial_step<K0, K1, K2, RK>(S, x, p, F, P.atol, P.rtol, tmax);
        }
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
    d[QCAMS_F_H * ld + i] = h;
    nstep[i] = 0;
    nrej[i] = 0;
    status[i] = st;
    if (sample)
        for (int f = 0; f < 6; ++f) sample[f * ld + i] = smp[f];
}

// ---------------------------------------------------------------------------
// propagation: one trajectory per lane until it stops
// ---------------------------------------------------------------------------
template <int K0, int K1, int K2, int RK>
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
        L.h = initial_step<K0, K1, K2, RK>(S, L.x, L.p, L.F, P.atol, P.rtol, L.tmax - L.t);
    if (!is_finite(L.t) || !is_finite(L.tmax) || !is_finite(L.h)) L.status = FAIL_NONFINITE;
    else if (L.t >= L.tmax) L.status = OK_TMAX;
    else if (L.nstep >= P.max_steps) L.status = FAIL_MAXSTEPS;
    while (L.status == RUNNING) lane_step<K0, K1, K2, RK>(S, P, L);
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
// propagation with a record of the pair distances: the same steps as
// k_propagate (one lane per trajectory, the same step function, so the same
// trajectory), writing (t, r_AB, r_BC, r_CA) at the start and after every
// accepted step into rec[i][0..rec_max), and the number written into rec_n.
// Past rec_max points the trajectory continues unrecorded.
// ---------------------------------------------------------------------------
__device__ inline void record_point(const Sys& S, const Lane& L, double* r)
{
    double ab = 0.0, bc = 0.0, ca = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double x1 = L.x[a], x2 = L.x[3 + a];
        const double u = x2 - S.cA * x1, w = -x2 - S.cB * x1;
        ab += x1 * x1;
        bc += u * u;
        ca += w * w;
    }
    r[0] = L.t;
    r[1] = sqrt(ab);
    r[2] = sqrt(bc);
    r[3] = sqrt(ca);
}

template <int K0, int K1, int K2, int RK>
__global__ void __launch_bounds__(256) k_record(Sys S, Prm P, double* d, int32_t* nstep,
                                                int32_t* nrej, uint8_t* status, int64_t ld,
                                                int64_t n, double* rec, int32_t rec_max,
                                                int32_t* rec_n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double* out = rec + i * (int64_t)rec_max * 4;
    int32_t m = 0;
    if (status[i] != RUNNING) {
        rec_n[i] = 0;
        return;
    }
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
        L.h = initial_step<K0, K1, K2, RK>(S, L.x, L.p, L.F, P.atol, P.rtol, L.tmax - L.t);
    if (!is_finite(L.t) || !is_finite(L.tmax) || !is_finite(L.h)) L.status = FAIL_NONFINITE;
    else if (L.t >= L.tmax) L.status = OK_TMAX;
    else if (L.nstep >= P.max_steps) L.status = FAIL_MAXSTEPS;
    if (m < rec_max) record_point(S, L, out + 4 * m++);
    while (L.status == RUNNING) {
        const int32_t before = L.nstep;
        lane_step<K0, K1, K2, RK>(S, P, L);
        if (L.nstep != before && m < rec_max) record_point(S, L, out + 4 * m++);
    }
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
    rec_n[i] = m;
}

// ---------------------------------------------------------------------------
// persistent propagation with lane refill
//
// Work items w = 0..N-1 are trajectories in longest-expected-first instance
// order.  Each slot (a lane, quad or octet) holds one trajectory; when at
// least `refill_min` slots of a wave are idle, lane 0 claims that many items
// of a work list with one atomic add and the idle slots take consecutive
// items of the list by their rank among the idle slots (ballot + mbcnt).  A
// slot picks up its trajectory's initial state (drawn beforehand by the
// initial-condition kernel) and writes the final state back to the same
// natural position (instances in id order), where classification and
// reduction read them.
// ---------------------------------------------------------------------------
// Work of the persistent run, XCD by XCD.  Each XCD (its own L2) has a list
// of its own: the work order cut into chunks of kChunk consecutive items,
// chunk k on list k mod kLists.  Consecutive items of an instance sit at
// consecutive natural positions, so the cache lines of a chunk's state rows
// are read and written by one XCD only.  A wave takes work from its XCD's
// list first and from the next lists once that one is used up.
constexpr int kChunk = 16;    // items per chunk: one 128-byte line of a state row
constexpr int kLists = 8;     // XCDs of the MI355X
constexpr int kWaveSteps = kLists;   // counter slot of the wave-step count
constexpr int kCounters = kLists + 1;

__global__ void k_reset_counter(unsigned long long* c)
{
    if (threadIdx.x < kCounters) c[threadIdx.x] = 0ull;
}

struct RunMap {
    const int64_t* order;   // work item -> natural position
    int64_t N;
};

// length of list x, and its j-th work item
__device__ inline int64_t list_len(int64_t N, int x)
{
    const int64_t full = N / (kChunk * kLists), rem = N % (kChunk * kLists);
    const int64_t tail = rem - (int64_t)x * kChunk;
    return full * kChunk + (tail < 0 ? 0 : (tail > kChunk ? kChunk : tail));
}

__device__ inline int64_t list_item(int64_t j, int x)
{
    return ((j / kChunk) * kLists + x) * kChunk + (j % kChunk);
}

// natural positions and ids of the installed instances, and the work order
// (instances longest-expected-first, or in id order)
__global__ void k_run_tables(const Inst* inst, int n_inst, const int32_t* ord_inst,
                             const int64_t* ord_off, const int64_t* nat_off, int64_t n,
                             int64_t* ids, int64_t* order)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= n) return;
    int lo = 0, hi = n_inst - 1, j = 0;
    while (lo <= hi) {   // last rank with ord_off <= w
        const int mid = (lo + hi) >> 1;
        if (ord_off[mid] <= w) { j = mid; lo = mid + 1; }
        else hi = mid - 1;
    }
    const int k = ord_inst[j];
    const int64_t local = w - ord_off[j];
    const int64_t pos = nat_off[k] + local;
    order[w] = pos;
    ids[pos] = inst[k].first_id + local;
}

// Makes a wave-uniform value opaque to the optimiser at this point, so that
// what is computed from it stays where it is written.
template <class T>
__device__ inline void opaque_sgpr(T& v)
{
    asm volatile("" : "+s"(v));
}

// A trajectory's slot is one lane (W = 1) or a quad of lanes (W = 4, see the
// lane layouts of the device header); the idle-slot count and a slot's rank
// among the idle slots are the lane counts divided by W.
template <int W>
__device__ inline void load_traj(const double* d, int64_t ld, int64_t pos, int c, int side,
                                 LaneW<W>& L)
{
    if constexpr (W == 1) {
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            L.x[f] = d[f * ld + pos];
            L.p[f] = d[(6 + f) * ld + pos];
        }
    } else if constexpr (W == 8) {
        // first quad: (rho1_c, P1_c); second quad: (rho2_c, P2_c)
        if (c < 3) {
            L.x[0] = d[(3 * side + c) * ld + pos];
            L.p[0] = d[(6 + 3 * side + c) * ld + pos];
        } else {
            L.x[0] = L.p[0] = 0.0;
        }
    } else {
        if (c < 3) {
            L.x[0] = d[c * ld + pos];
            L.x[1] = d[(3 + c) * ld + pos];
            L.p[0] = d[(6 + c) * ld + pos];
            L.p[1] = d[(9 + c) * ld + pos];
        } else {
            L.x[0] = L.x[1] = L.p[0] = L.p[1] = 0.0;
        }
    }
}

template <int W>
__device__ inline void store_traj(double* d, int64_t ld, int64_t pos, int c, int side,
                                  const LaneW<W>& L)
{
    if constexpr (W == 1) {
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            d[f * ld + pos] = L.x[f];
            d[(6 + f) * ld + pos] = L.p[f];
        }
    } else if constexpr (W == 8) {
        if (c < 3) {
            d[(3 * side + c) * ld + pos] = L.x[0];
            d[(6 + 3 * side + c) * ld + pos] = L.p[0];
        }
    } else {
        if (c < 3) {
            d[c * ld + pos] = L.x[0];
            d[(3 + c) * ld + pos] = L.x[1];
            d[(6 + c) * ld + pos] = L.p[0];
            d[(9 + c) * ld + pos] = L.p[1];
        }
    }
}

template <int W, int K0, int K1, int K2, int RK>
__global__ void __launch_bounds__(256)
k_persistent(Sys S, Prm P, RunMap M, unsigned long long* counter, int refill_min, int check_every,
             double* d, int32_t* nstep, int32_t* nrej, uint8_t* status, int64_t ld)
{
    constexpr int SLOTS = 64 / W;
    const unsigned lane = __lane_id();
    const int c = W == 1 ? 0 : (int)(lane & 3u);
    const int side = W == 8 ? (int)((lane >> 2) & 1u) : 0;
    const Role R = with_table<RK>(make_role(S, c, side));
    const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    LaneW<W> L;
    int64_t pos = -1;
    bool active = false;
    unsigned wsteps = 0;   // iterations in which the wave stepped any slot
    int lists_left = kLists;   // work lists this wave has not found used up
    L.status = RUNNING;
    for (;;) {
        // ---- refill (wave-uniform) ----
        const unsigned long long idle = __ballot(!active);
        const int nidle = __popcll(idle) / W;
        const bool none_active = nidle == SLOTS;
        // one grab per refill from the current list; slots it leaves idle
        // (the list ran out) are filled from the next list on the next pass
        if (lists_left > 0 && nidle > 0 && (nidle >= refill_min || none_active)) {
            // the wave's XCD: hardware register XCC_ID, bits 3:0
            const int xcd = (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (kLists - 1));
            const int x = (xcd + kLists - lists_left) & (kLists - 1);
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(&counter[x], (unsigned long long)nidle);
            const unsigned lo32 = __builtin_amdgcn_readfirstlane((unsigned)(base & 0xffffffffull));
            const unsigned hi32 = __builtin_amdgcn_readfirstlane((unsigned)(base >> 32));
            base = ((unsigned long long)hi32 << 32) | lo32;
            const int64_t left = list_len(M.N, x) - (int64_t)base;
            if (left < nidle) --lists_left;
            const int rank = __popcll(idle & lt_mask) / W;   // among the idle slots
            if (!active && rank < left) {
                const int64_t w = list_item((int64_t)base + rank, x);
                {
                    // row addresses formed here, not hoisted out of the loop
                    // (they would hold scalar registers across the steps)
                    const double* dr = d;
                    int64_t l = ld;
                    opaque_sgpr(dr);
                    opaque_sgpr(l);
                    pos = M.order[w];
                    load_traj<W>(dr, l, pos, c, side, L);
                    L.t = dr[QCAMS_F_T * l + pos];
                    L.tmax = dr[QCAMS_F_TMAX * l + pos];
                    const double rs = dr[QCAMS_F_RSTOP * l + pos];
                    L.rstop2 = rs * rs;
                    L.h = dr[QCAMS_F_H * l + pos];
                    L.nstep = nstep[pos];
                    L.nrej = nrej[pos];
                    L.last_rej = 0;
                    L.status = status[pos];
                    if (L.status == RUNNING) {
                        double s2[3];
                        force_w<W, K0, K1, K2>(S, R, L.x, L.F, s2);
                        if (!is_finite(L.t) || !is_finite(L.tmax) || !is_finite(L.h)) L.status = FAIL_NONFINITE;
                        else if (L.t >= L.tmax) L.status = OK_TMAX;
                        else if (L.nstep >= P.max_steps) L.status = FAIL_MAXSTEPS;
                    }
                    active = true;
                }
            }
        }
        if (__ballot(active) == 0ull) {
            if (lists_left == 0) break;
            continue;   // every slot idle: take from the next list at once
        }
        // ---- integrate ----
        const int32_t trials0 = L.nstep + L.nrej;
        for (int s = 0; s < check_every; ++s) {
            if (active && L.status == RUNNING) lane_step_w<W, K0, K1, K2, RK>(S, R, P, L);
        }
        // a slot that stops stays stopped until the retirement below, so the
        // iterations in which the wave stepped any slot are the most trials
        // one slot made; nearly always some slot made all of them
        {
            const int32_t ran = L.nstep + L.nrej - trials0;
            int k = check_every;
            while (k > 0 && __ballot(ran >= k) == 0ull) --k;
            wsteps += (unsigned)k;
        }
        // ---- retire finished trajectories ----
        if (active && L.status != RUNNING) {
            double* dw = d;
            int64_t l = ld;
            opaque_sgpr(dw);
            opaque_sgpr(l);
            store_traj<W>(dw, l, pos, c, side, L);
            if (c == 0 && side == 0) {
                dw[QCAMS_F_T * l + pos] = L.t;
                dw[QCAMS_F_H * l + pos] = L.h;
                nstep[pos] = L.nstep;
                nrej[pos] = L.nrej;
                status[pos] = (uint8_t)L.status;
            }
            active = false;
            L.status = RUNNING;
        }
    }
    if (lane == 0) atomicAdd(&counter[kWaveSteps], (unsigned long long)wsteps);
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
// per-instance reduction: 256-thread blocks over chunks of positions, fixed order
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

// The reduction of an instance runs in chunks of kXChunk positions, one
// block per chunk, each writing a row of partial sums; a second kernel adds
// an instance's rows in chunk order.  Both orders are fixed, so the results
// do not depend on timing, and an instance that fits in one chunk gets the
// sums a single block would form.
constexpr int64_t kXChunk = 4096;
constexpr int kPartHist = 3 * QCAMS_VMAX;     // (channel q, r1, r2) x v_t
constexpr int kPartStride = 16 + kPartHist;   // 16 sums, then the histogram

// ---------------------------------------------------------------------------
// Static scratch of the run without allocation (qcams_run_noalloc): the
// work-list counters, the work order and the reduction's partial sums of one
// run live in this file-scope device array, one copy per GPU (held until the
// process ends).  Host code never passes the array's name to a kernel (on
// the host it is only a stand-in for the symbol): each device's address is
// taken once with hipGetSymbolAddress, with that device current, when the
// first context on it is created, and kept in g_scratch_ptr.
// ---------------------------------------------------------------------------
constexpr int64_t kScratchItems = int64_t(1) << 21;   // trajectories per run
constexpr int64_t kScratchChunks = 8192;              // reduction chunks per run
constexpr size_t kScratchCounterBytes = 256;
constexpr size_t kScratchOrderOff = kScratchCounterBytes;
constexpr size_t kScratchPartOff = kScratchOrderOff + (size_t)kScratchItems * sizeof(int64_t);
constexpr size_t kScratchBytes = kScratchPartOff + (size_t)kScratchChunks * kPartStride * sizeof(double);
static_assert(kCounters * sizeof(unsigned long long) <= kScratchCounterBytes, "counter block");
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char* g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on `device` (which must be current), taken once.
static hipError_t scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = (unsigned char*)ptr;
    return hipSuccess;
}

static unsigned char* scratch_of(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    return g_scratch_ptr[device];
}

__device__ inline int instance_of_chunk(const int64_t* xoff, int n_inst, int64_t blk)
{
    int lo = 0, hi = n_inst - 1, k = 0;
    while (lo <= hi) {   // last instance whose first chunk is <= blk
        const int mid = (lo + hi) >> 1;
        if (xoff[mid] <= blk) { k = mid; lo = mid + 1; }
        else hi = mid - 1;
    }
    return k;
}

__global__ void __launch_bounds__(kRedThreads)
k_xsec_part(const Inst* inst, int n_inst, const int64_t* xoff, const uint8_t* label,
            const int16_t* vt, const double* od, int64_t old, const int64_t* ids,
            const double* weight, int64_t n, double* part)
{
    const int64_t blk = blockIdx.x;
    const int k = instance_of_chunk(xoff, n_inst, blk);
    __shared__ double red[16 * kRedThreads];
    const Inst I = inst[k];
    const int64_t ib = lower_bound_ids(ids, n, I.first_id);
    const int64_t ie = lower_bound_ids(ids, n, I.first_id + I.n_traj);
    const int64_t b = ib + (blk - xoff[k]) * kXChunk;
    const int64_t e = b + kXChunk < ie ? b + kXChunk : ie;
    double* row = part + blk * kPartStride;
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
    if (threadIdx.x < 16) row[threadIdx.x] = acc[threadIdx.x];
    // max-reduce through the same buffer
    red[threadIdx.x] = vtmax;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const int vmax_here = (int)fmin(red[0], (double)(QCAMS_VMAX - 1));
    __syncthreads();
    // Gaussian-binning histogram, one fixed-order reduction per (channel, vt)
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
            if (threadIdx.x == 0) row[16 + c * QCAMS_VMAX + v] = h[0];
        }
        for (int v = vmax_here + 1 + (int)threadIdx.x; v < QCAMS_VMAX; v += kRedThreads)
            row[16 + c * QCAMS_VMAX + v] = 0.0;
    }
}

__global__ void __launch_bounds__(kRedThreads)
k_xsec(const Inst* inst, int n_inst, const int64_t* xoff, const double* part, double mu123,
       const int64_t* ids, int64_t n, double* xs, double* hist)
{
    const int k = blockIdx.x;
    if (k >= n_inst) return;
    __shared__ double tot[kPartStride];
    // each sum over the instance's chunks in chunk order
    for (int q = threadIdx.x; q < kPartStride; q += kRedThreads) {
        double t = 0.0;
        for (int64_t r = xoff[k]; r < xoff[k + 1]; ++r) t += part[r * kPartStride + q];
        tot[q] = t;
    }
    __syncthreads();
    if (hist)
        for (int q = threadIdx.x; q < kPartHist; q += kRedThreads)
            hist[(int64_t)k * kPartHist + q] = tot[16 + q];
    if (threadIdx.x != 0) return;
    const Inst I = inst[k];
    const int64_t b = lower_bound_ids(ids, n, I.first_id);
    const int64_t e = lower_bound_ids(ids, n, I.first_id + I.n_traj);
    const double* acc = tot;
    double Wsum = 0.0;
    for (int q = 0; q < kPartHist; ++q) Wsum += tot[16 + q];
    double* row = xs + (int64_t)k * QCAMS_XS_STRIDE;
    const double N = (double)(e - b);
    row[0] = N;
    for (int c = 0; c < 6; ++c) row[1 + c] = acc[c];
    const double area = I.b_mode != QCAMS_B_FIXED ? kPi * I.bmax * I.bmax : NAN;
    const double speed = sqrt(2.0 * I.Ec / mu123);
    for (int c = 0; c < 4; ++c) {
        const double m = N > 0 ? acc[6 + c] / N : NAN;
        // m^2 rounded on its own (not fused into the difference): a single
        // trajectory, or all-equal weights, then give a variance of exactly 0
        const double m2 = m * m;
        const double var = N > 0 ? acc[10 + c] / N - m2 : NAN;
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
// Eq. (18)-(19) on fixed impact-parameter grids: per group of fixed-b
// instances with the same (E_c, v, j), ordered by b, sigma_x = 2 pi int P_x b db
// by the trapezoid rule over the grid (the reading 2 pi of the prefactor; b
// from the first to the last grid point), its error from the independent
// per-b errors, and the rate k_x = sigma_x sqrt(2 E_c / mu_123).  One thread
// per group.
// ---------------------------------------------------------------------------
__global__ void k_grid_xs(const Inst* inst, const int32_t* gidx, const int32_t* goff, int n_groups,
                          double mu123, const double* xs, double* out)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_groups) return;
    const int b0 = goff[g], b1 = goff[g + 1];
    double sig[4] = {0, 0, 0, 0}, var[4] = {0, 0, 0, 0}, N = 0.0;
    for (int q = b0; q < b1; ++q) {
        const int k = gidx[q];
        const double b = inst[k].b;
        const double lo = q > b0 ? inst[gidx[q - 1]].b : b;
        const double hi = q + 1 < b1 ? inst[gidx[q + 1]].b : b;
        const double w = 0.5 * (hi - lo);                // trapezoid weight of this node
        const double* row = xs + (int64_t)k * QCAMS_XS_STRIDE;
        N += row[0];
        for (int c = 0; c < 4; ++c) {
            const double f = w * (2.0 * kPi * b);
            sig[c] += f * row[7 + c];
            var[c] += (f * row[11 + c]) * (f * row[11 + c]);
        }
    }
    const Inst& I = inst[gidx[b0]];
    double* o = out + (int64_t)g * QCAMS_GRID_STRIDE;
    o[0] = I.Ec_K;
    o[1] = I.v;
    o[2] = I.j;
    o[3] = b1 - b0;
    o[4] = inst[gidx[b1 - 1]].b;
    o[5] = N;
    const double speed = sqrt(2.0 * I.Ec / mu123);
    for (int c = 0; c < 4; ++c) {
        o[6 + c] = sig[c];
        o[10 + c] = sqrt(var[c]);
        o[14 + c] = sig[c] * speed;
    }
    for (int c = 18; c < QCAMS_GRID_STRIDE; ++c) o[c] = 0.0;
}

// ---------------------------------------------------------------------------
// learned proposal: network inputs, cell table, cumulative distribution
// ---------------------------------------------------------------------------
constexpr double kFeatB = 10.0;   // impact parameter scale of the input (a0)

__device__ inline void features(double Ec_hartree, double b, int v, int j, double chi, double cth,
                                float* x)
{
    const double EK = Ec_hartree / 3.1668115634556e-6;
    x[0] = (float)((log10(EK) - 3.0) * 0.5);
    x[1] = (float)(b / kFeatB);
    x[2] = (float)(v * 0.1);
    x[3] = (float)(j * 0.1);
    x[4] = (float)chi;
    x[5] = (float)cth;
}

__global__ void k_mlp_features(const Inst* inst, int n_inst, const int64_t* ids, const double* sample,
                               int64_t sld, const uint8_t* label, int64_t n, float* x, int32_t* y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int k = find_instance(inst, n_inst, ids[i]);
    float f[6] = {0, 0, 0, 0, 0, 0};
    int lab = -1;
    if (k >= 0) {
        const Inst I = inst[k];
        features(I.Ec, sample[0 * sld + i], I.v, I.j, sample[4 * sld + i], sample[1 * sld + i], f);
        lab = label[i] < 4 ? (int)label[i] : -1;
    }
    for (int c = 0; c < 6; ++c) x[i * 6 + c] = f[c];
    y[i] = lab;
}

__global__ void k_cell_features(const Inst* inst, int k, float* x)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= kCells) return;
    const Inst I = inst[k];
    const int ib = c / (kCellsChi * kCellsCos), ichi = (c / kCellsCos) % kCellsChi, ic = c % kCellsCos;
    const double b = I.bmax * sqrt((ib + 0.5) / kCellsB);
    const double chi = (ichi + 0.5) / kCellsChi;
    const double cth = -1.0 + (ic + 0.5) * (2.0 / kCellsCos);
    features(I.Ec, b, I.v, I.j, chi, cth, x + 6 * c);
}

// q_k = alpha / K + (1 - alpha) sqrt(pi_k) / sum sqrt(pi); one block, fixed
// summation order.  With prob == NULL, q_k = 1/K.
__global__ void __launch_bounds__(256) k_prop_q(const float* prob, int channel, double alpha, double* q)
{
    __shared__ double part[256];
    const int t = threadIdx.x;
    constexpr int per = kCells / 256;
    double s = 0.0;
    for (int e = 0; e < per; ++e) {
        const int c = t * per + e;
        s += prob ? sqrt(fmax((double)prob[4 * c + channel], 0.0)) : 0.0;
    }
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        double tot = 0.0;
        for (int u = 0; u < 256; ++u) tot += part[u];
        part[0] = tot;
    }
    __syncthreads();
    const double tot = part[0];
    for (int e = 0; e < per; ++e) {
        const int c = t * per + e;
        const double r = (prob && tot > 0.0) ? sqrt(fmax((double)prob[4 * c + channel], 0.0)) / tot : 0.0;
        q[c] = (prob && tot > 0.0 && alpha < 1.0) ? alpha / kCells + (1.0 - alpha) * r : 1.0 / kCells;
    }
}

// normalised cumulative distribution of q (fixed order: 256 chunks of 32)
__global__ void __launch_bounds__(256) k_prop_cdf(double* q, double* cdf)
{
    __shared__ double part[257];
    const int t = threadIdx.x;
    constexpr int per = kCells / 256;
    double s = 0.0;
    for (int e = 0; e < per; ++e) s += q[t * per + e];
    part[t + 1] = s;
    __syncthreads();
    if (t == 0) {
        part[0] = 0.0;
        for (int u = 1; u <= 256; ++u) part[u] += part[u - 1];
    }
    __syncthreads();
    const double tot = part[256];
    double run = part[t];
    for (int e = 0; e < per; ++e) {
        const int c = t * per + e;
        run += q[c];
        cdf[c] = run / tot;
    }
    __syncthreads();
    for (int e = 0; e < per; ++e) q[t * per + e] /= tot;
    if (t == 255) cdf[kCells - 1] = 1.0;
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

// Units and reduced masses of the system (Sec. 3.1; Eq. (2)) and the pair
// parameters of the input forms: masses in electron masses, Morse range from
// the harmonic frequency, LJ coefficients from the depth and position of the
// minimum.  Returns 0, or -1 with a message.
static const double kAmuInMe = 1822.888486209;   // m_u / m_e, CODATA 2018
static int resolve_system(const qcams_system* in, qcams_system* out, char* msg, size_t len)
{
    qcams_system r = *in;
    if (in->mass_unit != QCAMS_MASS_ME && in->mass_unit != QCAMS_MASS_AMU) {
        snprintf(msg, len, "unknown mass unit %d", in->mass_unit);
        return -1;
    }
    for (int i = 0; i < 3; ++i) {
        if (!(in->mass[i] > 0.0)) {
            snprintf(msg, len, "mass %d must be > 0", i);
            return -1;
        }
        r.mass[i] = in->mass_unit == QCAMS_MASS_AMU ? in->mass[i] * kAmuInMe : in->mass[i];
    }
    r.mass_unit = QCAMS_MASS_ME;
    for (int i = 0; i < 3; ++i) {
        qcams_pair& q = r.pair[i];
        if (q.kind == QCAMS_MORSE_WE) {
            // alpha = w_e sqrt(mu / (2 De)), mu the pair's reduced mass
            const double ma = r.mass[i], mb = r.mass[(i + 1) % 3];
            const double mu = 1.0 / (1.0 / ma + 1.0 / mb);
            if (!(q.p[0] > 0.0) || !(q.p[2] > 0.0)) {
                snprintf(msg, len, "pair %d: Morse needs De > 0 and w_e > 0", i);
                return -1;
            }
            q.kind = QCAMS_MORSE;
            q.p[2] = q.p[2] * sqrt(mu / (2.0 * q.p[0]));
        } else if (q.kind == QCAMS_LJ_EPS) {
            // depth eps at r_m: Cn = eps m r_m^n / (n - m), Cm = eps n r_m^m / (n - m)
            const int n = q.n, m = q.m;
            const double eps = q.p[0], rm = q.p[1];
            if (!(n > m && m >= 3 && n <= 64) || !(eps > 0.0) || !(rm > 0.0)) {
                snprintf(msg, len, "pair %d: LJ needs n > m >= 3, eps > 0, r_m > 0", i);
                return -1;
            }
            q.kind = QCAMS_LJ;
            q.p[0] = eps * m * pow(rm, n) / (n - m);
            q.p[1] = eps * n * pow(rm, m) / (n - m);
        }
        if (!pair_ok(q)) {
            snprintf(msg, len, "pair %d: unsupported kind or parameters", i);
            return -1;
        }
    }
    *out = r;
    return 0;
}

// Kernels are specialised for the all-Morse and the LJ 12-6 / Morse /
// Buckingham pair triples (other triples select the pair kind at run time)
// and for the RK variant; `with_kinds` maps the context to the instantiation.
template <template <int, int, int, int> class L, int RK, class... A>
static void with_kinds(const qcams_ctx* c, A&&... a)
{
    if (c->kinds == 0) L<0, 0, 0, RK>::go(a...);
    else if (c->kinds == QCAMS_LJ + 3 * QCAMS_MORSE + 9 * QCAMS_BUCK && c->lj126)
        L<LJ126, 0, 2, RK>::go(a...);
    else L<-1, -1, -1, RK>::go(a...);
}

template <template <int, int, int, int> class L, class... A>
static void with_variant(const qcams_ctx* c, int rk, A&&... a)
{
    if (rk == 1) with_kinds<L, 1>(c, a...);
    else with_kinds<L, 0>(c, a...);
}

template <int K0, int K1, int K2, int RK>
struct PropagateL {
    static void go(qcams_ctx* c, const qcams_state* st, int64_t n, hipStream_t s)
    {
        hipLaunchKernelGGL((k_propagate<K0, K1, K2, RK>), dim3(grid_of(n, 256)), dim3(256), 0, s,
                           c->sys, c->prm, st->d, st->nstep, st->nrej, st->status, st->ld, n);
    }
};

template <int K0, int K1, int K2, int RK>
struct RecordL {
    static void go(qcams_ctx* c, const qcams_state* st, int64_t n, double* rec, int32_t rec_max,
                   int32_t* rec_n, hipStream_t s)
    {
        hipLaunchKernelGGL((k_record<K0, K1, K2, RK>), dim3(grid_of(n, 64)), dim3(64), 0, s, c->sys,
                           c->prm, st->d, st->nstep, st->nrej, st->status, st->ld, n, rec, rec_max,
                           rec_n);
    }
};

template <int K0, int K1, int K2, int RK>
struct PersistentL {
    static void go(qcams_ctx* c, int width, int blocks, int refill_min, int check_every,
                   const int64_t* order, unsigned long long* counter, const qcams_state* st,
                   hipStream_t s)
    {
        RunMap M{order, c->n_total};
        Prm P = c->prm;
        P.rk = RK;
        if (width == 8)
            hipLaunchKernelGGL((k_persistent<8, K0, K1, K2, RK>), dim3(blocks), dim3(256), 0, s,
                               c->sys, P, M, counter, refill_min, check_every, st->d,
                               st->nstep, st->nrej, st->status, st->ld);
        else if (width == 4)
            hipLaunchKernelGGL((k_persistent<4, K0, K1, K2, RK>), dim3(blocks), dim3(256), 0, s,
                               c->sys, P, M, counter, refill_min, check_every, st->d,
                               st->nstep, st->nrej, st->status, st->ld);
        else
            hipLaunchKernelGGL((k_persistent<1, K0, K1, K2, RK>), dim3(blocks), dim3(256), 0, s,
                               c->sys, P, M, counter, refill_min, check_every, st->d,
                               st->nstep, st->nrej, st->status, st->ld);
    }
};

template <int K0, int K1, int K2, int RK>
struct InitL {
    static void go(qcams_ctx* c, const int64_t* ids, int64_t n, const qcams_state* st,
                   double* sample, hipStream_t s)
    {
        Prm P = c->prm;
        P.rk = RK;
        hipLaunchKernelGGL((k_init<K0, K1, K2, RK>), dim3(grid_of(n, 256)), dim3(256), 0, s, c->sys,
                           P, c->d_inst, c->n_inst, ids, n, st->d, st->nstep, st->nrej, st->status,
                           st->ld, sample, (const double*)c->d_prop_q, (const double*)c->d_prop_cdf);
    }
};

static void dispatch_init(qcams_ctx* c, int rk, const int64_t* ids, int64_t n,
                          const qcams_state* st, double* sample, hipStream_t s)
{
    with_variant<InitL>(c, rk, c, ids, n, st, sample, s);
}

extern "C" {

int qcams_system_resolve(const qcams_system* in, qcams_system* out)
{
    if (!in || !out) return fail(nullptr, QCAMS_EINVAL, "null argument");
    char msg[256];
    if (resolve_system(in, out, msg, sizeof msg) != 0) return fail(nullptr, QCAMS_EINVAL, "%s", msg);
    return QCAMS_OK;
}

int qcams_create(qcams_ctx** out, int device, const qcams_system* sys_in, const qcams_params* prm)
{
    if (!out || !sys_in || !prm) return fail(nullptr, QCAMS_EINVAL, "null argument");
    *out = nullptr;
    qcams_system resolved;
    {
        char msg[256];
        if (resolve_system(sys_in, &resolved, msg, sizeof msg) != 0)
            return fail(nullptr, QCAMS_EINVAL, "%s", msg);
    }
    const qcams_system* sys = &resolved;
    if (!(prm->atol > 0.0) || !(prm->rtol >= 0.0) || !(prm->t_stop > 0.0) || !(prm->r_stop > 0.0) ||
        !(prm->R0 > 0.0) || !(prm->gb_sigma > 0.0) || prm->max_steps < 1 ||
        prm->max_steps > 2147483647LL || (prm->fixed_step && !(prm->h_fixed > 0.0)) ||
        (prm->rk != 0 && prm->rk != 1))
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
    {
        // per device, once: the static scratch of qcams_run_noalloc, the
        // compute-unit count and the events around the persistent launch
        hipError_t e = scratch_setup(device);
        int cu = 0;
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device);
        c->n_cu = cu > 0 ? cu : 256;
        for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreate(&c->ev_prop[k]);
        if (e != hipSuccess) {
            for (int k = 0; k < 2; ++k)
                if (c->ev_prop[k]) (void)hipEventDestroy(c->ev_prop[k]);
            delete c;
            return fail(nullptr, QCAMS_EHIP, "device set-up: %s", hipGetErrorString(e));
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
        qcams_destroy(c);
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
        qcams_destroy(c);
        return fail(nullptr, QCAMS_EHIP, "pair shapes: %s", hipGetErrorString(e));
    }
    for (int i = 0; i < 3; ++i) {
        if (pot_is_zero(sys->pair[i])) {
            h_sh[i] = Shape{0.0, sys->pair[i].p[1], 2.0 * sys->pair[i].p[1], 0.0};
            continue;
        }
        if (h_rc[i] != 0) {
            qcams_destroy(c);
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
    c->lj126 = S.pot[0].kind == QCAMS_LJ && S.pot[0].n == 12 && S.pot[0].m == 6;
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
    c->prm.rk = prm->rk;
    c->prm.pad = 0;
    *out = c;
    return rc;
}

void qcams_destroy(qcams_ctx* c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->graph2_exec) (void)hipGraphExecDestroy(c->graph2_exec);
    if (c->graph2) (void)hipGraphDestroy(c->graph2);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->d_inst) (void)hipFree(c->d_inst);
    if (c->d_lpt_inst) (void)hipFree(c->d_lpt_inst);
    if (c->d_id_inst) (void)hipFree(c->d_id_inst);
    if (c->d_lpt_off) (void)hipFree(c->d_lpt_off);
    if (c->d_nat_off) (void)hipFree(c->d_nat_off);
    if (c->d_counter) (void)hipFree(c->d_counter);
    if (c->d_order) (void)hipFree(c->d_order);
    for (int e = 0; e < 2; ++e)
        if (c->ev_prop[e]) (void)hipEventDestroy(c->ev_prop[e]);
    for (void* q : {(void*)c->d_prop_q, (void*)c->d_prop_cdf, (void*)c->d_cell_x, (void*)c->d_cell_p,
                    (void*)c->d_grid_inst, (void*)c->d_grid_off, (void*)c->d_xoff, (void*)c->d_xpart})
        if (q) (void)hipFree(q);
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
        hipLaunchKernelGGL(k_levels, dim3(n), dim3(64), 0, 0, c->sys.pot[0],
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

int qd_dvr_eigenvalues(int device, const Pot& P, double mu, double a, double b, int n, int nj,
                       const int* js, int K, double* out, char* err, size_t errlen);

int qcams_dvr_levels(qcams_ctx* c, int32_t npts, double xmin, double xmax, int32_t n,
                     const int32_t* v, const int32_t* j, double* out)
{
    if (!c) return fail(nullptr, QCAMS_EINVAL, "null context");
    if (n < 0 || (n > 0 && (!v || !j || !out))) return fail(c, QCAMS_EINVAL, "bad arguments");
    if (npts < 16 || npts > 4096 || !(xmin > 0.0) || !(xmax > xmin))
        return fail(c, QCAMS_EINVAL, "DVR grid: need 16 <= npts <= 4096 and 0 < xmin < xmax");
    if (n == 0) return QCAMS_OK;
    std::vector<int> js;
    int K = 0;
    for (int i = 0; i < n; ++i) {
        if (v[i] < 0 || j[i] < 0) return fail(c, QCAMS_EINVAL, "negative quantum number");
        if (v[i] >= npts) return fail(c, QCAMS_EUNBOUND, "v=%d exceeds the DVR grid", v[i]);
        if (std::find(js.begin(), js.end(), j[i]) == js.end()) js.push_back(j[i]);
        K = std::max(K, v[i] + 1);
    }
    std::vector<double> eig((size_t)K * js.size());
    char msg[200] = {0};
    const int drc = qd_dvr_eigenvalues(c->device, c->sys.pot[0], c->sys.mu12, xmin, xmax, npts,
                                       (int)js.size(), js.data(), K, eig.data(), msg, sizeof msg);
    if (drc == -1) return fail(c, QCAMS_ENOMEM, "%s", msg);
    if (drc != 0) return fail(c, QCAMS_EHIP, "%s", msg);
    std::vector<double> E(n);
    for (int i = 0; i < n; ++i) {
        const size_t q = std::find(js.begin(), js.end(), j[i]) - js.begin();
        E[i] = eig[q * K + v[i]];
    }
    HIP_OK(c, hipSetDevice(c->device));
    int *dj = nullptr, *drc2 = nullptr;
    double *dE = nullptr, *dout = nullptr;
    std::vector<int> rc(n);
    hipError_t e = hipMalloc(&dj, n * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&drc2, n * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&dE, n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&dout, 4 * (size_t)n * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(dj, j, n * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dE, E.data(), n * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_levels_at, dim3(grid_of(n, 64)), dim3(64), 0, 0, c->sys.pot[0],
                           c->sys.shape[0], c->sys.mu12, n, (const double*)dE, (const int*)dj, dout,
                           drc2);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(out, dout, 4 * (size_t)n * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(rc.data(), drc2, n * sizeof(int), hipMemcpyDeviceToHost);
    for (void* q : {(void*)dj, (void*)drc2, (void*)dE, (void*)dout}) (void)hipFree(q);
    if (e != hipSuccess) return fail(c, QCAMS_EHIP, "DVR levels: %s", hipGetErrorString(e));
    for (int i = 0; i < n; ++i) {
        if (rc[i] == -2) return fail(c, QCAMS_EUNBOUND, "DVR level v=%d j=%d is not bound", v[i], j[i]);
        if (rc[i] != 0) return fail(c, QCAMS_ENOROOT, "DVR level v=%d j=%d: no turning points", v[i], j[i]);
    }
    return QCAMS_OK;
}

int qcams_set_level_method(qcams_ctx* c, int32_t method, int32_t npts, double xmin, double xmax)
{
    if (!c) return fail(nullptr, QCAMS_EINVAL, "null context");
    if (method == QCAMS_LEVELS_BS) {
        c->level_method = method;
        return QCAMS_OK;
    }
    if (method != QCAMS_LEVELS_DVR) return fail(c, QCAMS_EINVAL, "unknown level method");
    if (npts < 16 || npts > 4096 || !(xmin > 0.0) || !(xmax > xmin))
        return fail(c, QCAMS_EINVAL, "DVR grid: need 16 <= npts <= 4096 and 0 < xmin < xmax");
    c->level_method = method;
    c->dvr_npts = npts;
    c->dvr_xmin = xmin;
    c->dvr_xmax = xmax;
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
            (q.b_mode != QCAMS_B_FIXED && q.b_mode != QCAMS_B_AREA && q.b_mode != QCAMS_B_PROPOSAL) ||
            (q.b_mode == QCAMS_B_FIXED && !(q.b >= 0.0)) ||
            (q.b_mode != QCAMS_B_FIXED && !(q.bmax >= 0.0)))
            return fail(c, QCAMS_EINVAL, "instance %d: invalid fields", k);
        if (k > 0 && q.first_id < inst[k - 1].first_id + inst[k - 1].n_traj)
            return fail(c, QCAMS_EINVAL, "instance %d: ids overlap or are not sorted", k);
        // kelvin -> hartree (Boltzmann constant in E_h / K, CODATA 2018)
        h[k].Ec = q.Ec_K * 3.1668115634556e-6;
        h[k].Ec_K = q.Ec_K;
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
    // levels of the distinct (v, j) pairs only (instances share them: a grid
    // of energies repeats every state)
    std::vector<int32_t> uv, uj, which(n_inst);
    {
        std::map<std::pair<int32_t, int32_t>, int32_t> seen;
        for (int k = 0; k < n_inst; ++k) {
            const auto key = std::make_pair(vv[k], jj[k]);
            auto it = seen.find(key);
            if (it == seen.end()) {
                it = seen.emplace(key, (int32_t)uv.size()).first;
                uv.push_back(vv[k]);
                uj.push_back(jj[k]);
            }
            which[k] = it->second;
        }
    }
    const int n_lev = (int)uv.size();
    std::vector<double> lev(4 * (size_t)n_lev);
    int rc = c->level_method == QCAMS_LEVELS_DVR
                 ? qcams_dvr_levels(c, c->dvr_npts, c->dvr_xmin, c->dvr_xmax, n_lev, uv.data(),
                                    uj.data(), lev.data())
                 : qcams_levels(c, n_lev, uv.data(), uj.data(), lev.data());
    if (rc != QCAMS_OK) return rc;
    for (int k = 0; k < n_inst; ++k) {
        const double* L = &lev[4 * (size_t)which[k]];
        h[k].Evj = L[0];
        h[k].rminus = L[1];
        h[k].rplus = L[2];
        h[k].tau = L[3];
        const double b = inst[k].b_mode == QCAMS_B_FIXED ? inst[k].b : inst[k].bmax;
        if (!(b < c->prm.R0)) return fail(c, QCAMS_EINVAL, "instance %d: impact parameter >= R0", k);
    }
    HIP_OK(c, hipSetDevice(c->device));
    // device tables are reused while they are large enough, so that a captured
    // run (which reads them at replay time) stays valid
    if (n_inst > c->inst_cap) {
        for (void* q : {(void*)c->d_inst, (void*)c->d_lpt_inst, (void*)c->d_id_inst,
                        (void*)c->d_lpt_off, (void*)c->d_nat_off})
            if (q) (void)hipFree(q);
        c->d_inst = nullptr;
        c->d_lpt_inst = c->d_id_inst = nullptr;
        c->d_lpt_off = c->d_nat_off = nullptr;
        c->inst_cap = 0;
        c->n_inst = 0;
        c->graph_key[0] = 0;
        if (hipMalloc(&c->d_inst, n_inst * sizeof(Inst)) != hipSuccess ||
            hipMalloc(&c->d_lpt_inst, n_inst * sizeof(int32_t)) != hipSuccess ||
            hipMalloc(&c->d_id_inst, n_inst * sizeof(int32_t)) != hipSuccess ||
            hipMalloc(&c->d_lpt_off, (n_inst + 1) * sizeof(int64_t)) != hipSuccess ||
            hipMalloc(&c->d_nat_off, (n_inst + 1) * sizeof(int64_t)) != hipSuccess)
            return fail(c, QCAMS_ENOMEM, "instance table allocation failed");
        c->inst_cap = n_inst;
    }
    HIP_OK(c, hipMemcpy(c->d_inst, h.data(), n_inst * sizeof(Inst), hipMemcpyHostToDevice));
    c->n_inst = n_inst;
    c->h_inst = h;
    // fixed-b groups, keyed by (E_c, v, j) in order of first appearance
    {
        std::vector<std::vector<int32_t>> groups;
        std::vector<std::tuple<double, int, int>> keys;
        c->h_group_of.assign(n_inst, -1);
        for (int k = 0; k < n_inst; ++k) {
            if (inst[k].b_mode != QCAMS_B_FIXED) continue;
            const auto key = std::make_tuple(inst[k].Ec_K, inst[k].v, inst[k].j);
            int g = -1;
            for (size_t q = 0; q < keys.size(); ++q)
                if (keys[q] == key) { g = (int)q; break; }
            if (g < 0) {
                g = (int)keys.size();
                keys.push_back(key);
                groups.emplace_back();
            }
            groups[g].push_back(k);
            c->h_group_of[k] = g;
        }
        std::vector<int32_t> gidx, goff(1, 0);
        for (auto& m : groups) {
            std::stable_sort(m.begin(), m.end(),
                             [&](int32_t a, int32_t b) { return inst[a].b < inst[b].b; });
            gidx.insert(gidx.end(), m.begin(), m.end());
            goff.push_back((int32_t)gidx.size());
        }
        const int ng = (int)groups.size();
        if (ng > 0 && (int)gidx.size() + ng + 1 > c->grid_cap) {
            if (c->d_grid_inst) HIP_OK(c, hipFree(c->d_grid_inst));
            if (c->d_grid_off) HIP_OK(c, hipFree(c->d_grid_off));
            c->d_grid_inst = c->d_grid_off = nullptr;
            c->grid_cap = 0;
            if (hipMalloc(&c->d_grid_inst, gidx.size() * sizeof(int32_t)) != hipSuccess ||
                hipMalloc(&c->d_grid_off, (ng + 1) * sizeof(int32_t)) != hipSuccess)
                return fail(c, QCAMS_ENOMEM, "grid table allocation failed");
            c->grid_cap = (int)gidx.size() + ng + 1;
        }
        if (ng > 0) {
            HIP_OK(c, hipMemcpy(c->d_grid_inst, gidx.data(), gidx.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice));
            HIP_OK(c, hipMemcpy(c->d_grid_off, goff.data(), goff.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice));
        }
        c->n_groups = ng;
    }
    // natural offsets and the longest-expected-first order: expected trial
    // steps of a trajectory ~ collision time / step size, taken as
    // 1/(v_c sqrt(tau)): the step is set by the initial vibration (period
    // tau) for a light, stiff molecule, less so where the inner walls of an
    // anharmonic or heavy molecule set it; on the all-Morse and the mixed
    // surfaces this ranks the instances by their longest trajectories with
    // rank correlations 0.994 and 0.986 (1/(v_c tau): 0.995, 0.969)
    std::vector<int64_t> nat(n_inst + 1, 0), loff(n_inst + 1, 0);
    for (int k = 0; k < n_inst; ++k) nat[k + 1] = nat[k] + h[k].n_traj;
    // reduction chunks: at least one per instance
    {
        std::vector<int64_t> xoff(n_inst + 1, 0);
        for (int k = 0; k < n_inst; ++k) {
            const int64_t m = (h[k].n_traj + kXChunk - 1) / kXChunk;
            xoff[k + 1] = xoff[k] + (m > 0 ? m : 1);
        }
        const int64_t nch = xoff[n_inst];
        if (nch > 0x7fffffff) return fail(c, QCAMS_EINVAL, "too many reduction chunks");
        if (n_inst + 1 > c->xoff_cap || nch > c->xpart_cap) {
            if (c->d_xoff) (void)hipFree(c->d_xoff);
            if (c->d_xpart) (void)hipFree(c->d_xpart);
            c->d_xoff = nullptr;
            c->d_xpart = nullptr;
            c->xoff_cap = c->xpart_cap = 0;
            c->graph_key[0] = 0;
            if (hipMalloc(&c->d_xoff, (n_inst + 1) * sizeof(int64_t)) != hipSuccess ||
                hipMalloc(&c->d_xpart, nch * kPartStride * sizeof(double)) != hipSuccess)
                return fail(c, QCAMS_ENOMEM, "reduction table allocation failed");
            c->xoff_cap = n_inst + 1;
            c->xpart_cap = nch;
        }
        HIP_OK(c, hipMemcpy(c->d_xoff, xoff.data(), (n_inst + 1) * sizeof(int64_t),
                            hipMemcpyHostToDevice));
        c->n_xchunks = nch;
    }
    std::vector<int32_t> order(n_inst);
    std::vector<double> cost(n_inst);
    for (int k = 0; k < n_inst; ++k) {
        order[k] = k;
        const double vc = sqrt(2.0 * h[k].Ec * c->sys.inv_mu123);
        cost[k] = 1.0 / (vc * sqrt(h[k].tau));
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return cost[a] > cost[b]; });
    c->cost_max = 0.0;
    c->cost_total = 0.0;
    for (int k = 0; k < n_inst; ++k) {
        if (h[k].n_traj > 0) c->cost_max = std::max(c->cost_max, cost[k]);
        c->cost_total += cost[k] * (double)h[k].n_traj;
    }
    for (int r = 0; r < n_inst; ++r) loff[r + 1] = loff[r] + h[order[r]].n_traj;
    std::vector<int32_t> ident(n_inst);
    for (int k = 0; k < n_inst; ++k) ident[k] = k;
    c->n_total = nat[n_inst];
    HIP_OK(c, hipMemcpy(c->d_nat_off, nat.data(), (n_inst + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
    HIP_OK(c, hipMemcpy(c->d_lpt_off, loff.data(), (n_inst + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
    HIP_OK(c, hipMemcpy(c->d_lpt_inst, order.data(), n_inst * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_OK(c, hipMemcpy(c->d_id_inst, ident.data(), n_inst * sizeof(int32_t), hipMemcpyHostToDevice));
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
    dispatch_init(c, c->prm.rk, ids, n, st, sample, (hipStream_t)stream);
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
    with_variant<PropagateL>(c, c->prm.rk, c, st, n, s);
    HIP_OK(c, hipGetLastError());
    return QCAMS_OK;
}

int qcams_propagate_record(qcams_ctx* c, const qcams_state* st, int64_t n, double* rec,
                           int32_t rec_max, int32_t* rec_n, void* stream)
{
    if (!c) return fail(nullptr, QCAMS_EINVAL, "null context");
    if (int rc = check_state(c, st, n)) return rc;
    if (rec_max < 1 || (n > 0 && (!rec || !rec_n)))
        return fail(c, QCAMS_EINVAL, "record buffers missing or rec_max < 1");
    if (n == 0) return QCAMS_OK;
    HIP_OK(c, hipSetDevice(c->device));
    with_variant<RecordL>(c, c->prm.rk, c, st, n, rec, rec_max, rec_n, (hipStream_t)stream);
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

// the two reduction kernels: partial sums per chunk (rows of xpart), then
// per instance
static void launch_xsec(qcams_ctx* c, const qcams_outcome* out, const int64_t* ids,
                        const double* weight, int64_t n, double* xs, double* hist, double* xpart,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_xsec_part, dim3((unsigned)c->n_xchunks), dim3(kRedThreads), 0, s, c->d_inst,
                       c->n_inst, c->d_xoff, out->label, out->vt, out->d, out->ld, ids, weight, n,
                       xpart);
    hipLaunchKernelGGL(k_xsec, dim3(c->n_inst), dim3(kRedThreads), 0, s, c->d_inst, c->n_inst,
                       c->d_xoff, (const double*)xpart, c->sys.mu123, ids, n, xs, hist);
}

int qcams_cross_sections(qcams_ctx* c, const qcams_outcome* out, const int64_t* ids,
                         const double* weight, int64_t n, double* xs, double* hist, void* stream)
{
    if (!c) return fail(nullptr, QCAMS_EINVAL, "null context");
    if (c->n_inst < 1) return fail(c, QCAMS_EINVAL, "no instances installed");
    if (!out || !xs || n < 0 || (n > 0 && (!ids || !out->label || !out->vt || !out->d || out->ld < n)))
        return fail(c, QCAMS_EINVAL, "bad arguments");
    HIP_OK(c, hipSetDevice(c->device));
    launch_xsec(c, out, ids, weight, n, xs, hist, c->d_xpart, (hipStream_t)stream);
    HIP_OK(c, hipGetLastError());
    return QCAMS_OK;
}


// ---------------------------------------------------------------------------
// fused persistent run, launch-graph capture, autotuning
// ---------------------------------------------------------------------------
// RK variant of a run: the option overrides the context's parameter
static int run_variant(const qcams_ctx* c, const qcams_run_opts* o)
{
    return o->rk == 1 ? 0 : (o->rk == 2 ? 1 : c->prm.rk);
}

// Lanes per trajectory of the persistent kernel.  Default: an octet when
// every trajectory fits in the grid's octet slots at once (the run is then
// bound by its longest trajectory, and an octet step is about 5 % shorter
// than a quad's); otherwise from the expected step counts (~ 1/(v_c
// sqrt(tau)) per trajectory of an instance): the run is bound by its longest
// trajectory (C, allowing 1.5x for the spread inside an instance) or by its
// total work W over the L lanes of a one-lane grid.  A quad takes about
// half the time per step but gives half the throughput, so it is chosen
// when C > 2.1 W / L.
static int run_width(const qcams_ctx* c, const qcams_run_opts* o)
{
    if (o->lanes == 1 || o->lanes == 4 || o->lanes == 8) return o->lanes;
    const double L = 256.0 * (o->blocks > 0 ? o->blocks : c->n_cu);
    if (8.0 * (double)c->n_total <= L) return 8;
    return 1.5 * c->cost_max > 2.1 * c->cost_total / L ? 4 : 1;
}

// Device work buffers of one run: the work-list cursors and wave-step count
// [kCounters], the work order [n_total], the reduction's per-chunk partial
// sums [n_xchunks][kPartStride].  qcams_run uses the context's own
// allocations; qcams_run_noalloc the device's static scratch array.
struct RunBufs {
    unsigned long long* counter;
    int64_t* order;
    double* xpart;
};

// The run is three launch groups: the small set-up kernels (work order,
// initial conditions, counter reset), the persistent propagation kernel, and
// the small analysis kernels (classification, reduction).  In graph mode the
// two small groups are captured and replayed; the persistent kernel is one
// launch either way and is bracketed by HIP events for its duration.
static void enqueue_pre(qcams_ctx* c, const qcams_run_opts* o, const RunBufs& B,
                        const qcams_state* st, double* sample, int64_t* ids, hipStream_t s)
{
    const int64_t n = c->n_total;
    const bool lpt = o->lpt != 0;
    hipLaunchKernelGGL(k_run_tables, dim3(grid_of(n, 256)), dim3(256), 0, s, c->d_inst, c->n_inst,
                       lpt ? c->d_lpt_inst : c->d_id_inst, lpt ? c->d_lpt_off : c->d_nat_off,
                       c->d_nat_off, n, ids, B.order);
    dispatch_init(c, run_variant(c, o), ids, n, st, sample, s);
    // a fill kernel, not a memset: the counters start at zero also in
    // captured graphs
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, B.counter);
}

static int enqueue_persistent(qcams_ctx* c, const qcams_run_opts* o, const RunBufs& B,
                              const qcams_state* st, hipStream_t s)
{
    const int blocks = o->blocks > 0 ? o->blocks : c->n_cu;
    const int width = run_width(c, o);
    const int slots = 64 / width;
    const int rm = o->refill_min < 1 ? 1 : (o->refill_min > slots ? slots : o->refill_min);
    const int ce = o->check_every < 1 ? 1 : o->check_every;
    if (hipEventRecord(c->ev_prop[0], s) != hipSuccess) return QCAMS_EHIP;
    with_variant<PersistentL>(c, run_variant(c, o), c, width, blocks, rm, ce,
                              (const int64_t*)B.order, B.counter, st, s);
    c->last_counter = B.counter;
    c->last_opts = *o;
    c->last_opts.blocks = blocks;
    c->last_opts.refill_min = rm;
    c->last_opts.check_every = ce;
    c->last_opts.rk = run_variant(c, o) + 1;
    c->last_opts.lanes = width;
    c->last_opts.pad = 0;
    c->has_run = true;
    if (hipEventRecord(c->ev_prop[1], s) != hipSuccess) return QCAMS_EHIP;
    return hipGetLastError() == hipSuccess ? QCAMS_OK : QCAMS_EHIP;
}

static void enqueue_post(qcams_ctx* c, const RunBufs& B, const qcams_state* st,
                         const qcams_outcome* out, int64_t* ids, double* sample, double* xs,
                         double* hist, hipStream_t s)
{
    const int64_t n = c->n_total;
    hipLaunchKernelGGL(k_classify, dim3(grid_of(n, 128)), dim3(128), 0, s, c->sys, c->prm, st->d,
                       st->status, st->ld, n, out->label, out->vt, out->jt, out->d, out->ld);
    launch_xsec(c, out, ids, sample ? (const double*)(sample + 5 * st->ld) : (const double*)nullptr,
                n, xs, hist, B.xpart, s);
}

static int capture(qcams_ctx* c, hipGraph_t* g, hipGraphExec_t* x, const std::function<void(hipStream_t)>& f)
{
    if (*x) { HIP_OK(c, hipGraphExecDestroy(*x)); *x = nullptr; }
    if (*g) { HIP_OK(c, hipGraphDestroy(*g)); *g = nullptr; }
    if (!c->cap_stream) HIP_OK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIP_OK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    f(c->cap_stream);
    hipGraph_t gg = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &gg);
    if (e != hipSuccess) return fail(c, QCAMS_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    *g = gg;
    HIP_OK(c, hipGraphInstantiate(x, gg, nullptr, nullptr, 0));
    return QCAMS_OK;
}

// Arguments of a run (qcams_run, qcams_run_noalloc): buffers present and
// large enough, options valid; *o receives the options with defaults.
static int run_args(qcams_ctx* c, const qcams_run_opts* opts, const qcams_state* st,
                    const double* sample, const qcams_outcome* out, const int64_t* ids,
                    const double* xs, qcams_run_opts* o)
{
    if (c->n_inst < 1) return fail(c, QCAMS_EINVAL, "no instances installed");
    const int64_t n = c->n_total;
    if (int rc = check_state(c, st, n)) return rc;
    if (!out || !ids || !xs || (n > 0 && (!out->label || !out->vt || !out->jt || !out->d || out->ld < n)))
        return fail(c, QCAMS_EINVAL, "outcome / ids / xs buffers missing or too small");
    *o = qcams_run_opts{};
    o->blocks = 0;
    o->refill_min = 1;
    o->check_every = 8;
    o->lpt = 1;
    o->graph = 0;
    if (opts) *o = *opts;
    if (o->blocks < 0 || o->refill_min < 0 || o->check_every < 0 || o->rk < 0 || o->rk > 2 ||
        (o->lanes != 0 && o->lanes != 1 && o->lanes != 4 && o->lanes != 8))
        return fail(c, QCAMS_EINVAL, "invalid run option");
    for (const Inst& I : c->h_inst)
        if (I.b_mode == 2 && (!sample || !c->d_prop_q))
            return fail(c, QCAMS_EINVAL, "proposal instances need a sample buffer and a proposal");
    return QCAMS_OK;
}

int qcams_run(qcams_ctx* c, const qcams_run_opts* opts, const qcams_state* st, double* sample,
              const qcams_outcome* out, int64_t* ids, double* xs, double* hist, void* stream)
{
    if (!c) return fail(nullptr, QCAMS_EINVAL, "null context");
    qcams_run_opts o;
    if (int rc = run_args(c, opts, st, sample, out, ids, xs, &o)) return rc;
    const int64_t n = c->n_total;
    HIP_OK(c, hipSetDevice(c->device));
    if (!c->d_counter) {
        if (hipMalloc(&c->d_counter, kCounters * sizeof(unsigned long long)) != hipSuccess) {
            c->d_counter = nullptr;
            return fail(c, QCAMS_ENOMEM, "work list counters allocation failed");
        }
    }
    if (c->n_cu == 0) {
        int cu = 0;
        HIP_OK(c, hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, c->device));
        c->n_cu = cu > 0 ? cu : 256;
    }
    for (int e = 0; e < 2; ++e)
        if (!c->ev_prop[e]) HIP_OK(c, hipEventCreate(&c->ev_prop[e]));
    if (c->order_cap < n) {
        if (c->d_order) HIP_OK(c, hipFree(c->d_order));
        c->d_order = nullptr;
        c->order_cap = 0;
        if (hipMalloc(&c->d_order, (size_t)(n > 0 ? n : 1) * sizeof(int64_t)) != hipSuccess) {
            c->d_order = nullptr;
            return fail(c, QCAMS_ENOMEM, "work order allocation failed");
        }
        c->order_cap = n;
        c->graph_key[0] = 0;
    }
    hipStream_t s = (hipStream_t)stream;
    const RunBufs B{c->d_counter, c->d_order, c->d_xpart};
    if (!o.graph) {
        enqueue_pre(c, &o, B, st, sample, ids, s);
        if (enqueue_persistent(c, &o, B, st, s) != QCAMS_OK)
            return fail(c, QCAMS_EHIP, "run launch: %s", hipGetErrorString(hipGetLastError()));
        enqueue_post(c, B, st, out, ids, sample, xs, hist, s);
        HIP_OK(c, hipGetLastError());
        return QCAMS_OK;
    }
    // graph mode: capture the two small launch groups once per (buffers,
    // options, instance table, proposal tables), replay them around the
    // persistent launch; the kernels read the tables' contents at replay
    const uint64_t key[18] = {1,
                              (uint64_t)st->d, (uint64_t)st->nstep, (uint64_t)st->nrej,
                              (uint64_t)st->status, (uint64_t)st->ld, (uint64_t)sample,
                              (uint64_t)out->label, (uint64_t)out->d, (uint64_t)out->ld,
                              (uint64_t)ids, (uint64_t)xs, (uint64_t)hist,
                              (uint64_t)o.lpt | ((uint64_t)o.rk << 8) | ((uint64_t)c->n_xchunks << 16),
                              (uint64_t)out->vt ^ ((uint64_t)out->jt << 1),
                              (uint64_t)c->n_total ^ ((uint64_t)c->n_inst << 40),
                              (uint64_t)c->d_prop_q, (uint64_t)c->d_prop_cdf};
    if (memcmp(key, c->graph_key, sizeof key) != 0) {
        c->graph_key[0] = 0;
        int rc = capture(c, &c->graph, &c->graph_exec,
                         [&](hipStream_t cs) { enqueue_pre(c, &o, B, st, sample, ids, cs); });
        if (rc == QCAMS_OK)
            rc = capture(c, &c->graph2, &c->graph2_exec, [&](hipStream_t cs) {
                enqueue_post(c, B, st, out, ids, sample, xs, hist, cs);
            });
        if (rc != QCAMS_OK) return rc;
        memcpy(c->graph_key, key, sizeof key);
    }
    HIP_OK(c, hipGraphLaunch(c->graph_exec, s));
    if (enqueue_persistent(c, &o, B, st, s) != QCAMS_OK)
        return fail(c, QCAMS_EHIP, "run launch: %s", hipGetErrorString(hipGetLastError()));
    HIP_OK(c, hipGraphLaunch(c->graph2_exec, s));
    return QCAMS_OK;
}

int qcams_run_noalloc(qcams_ctx* c, const qcams_run_opts* opts, const qcams_state* st,
                      double* sample, const qcams_outcome* out, int64_t* ids, double* xs,
                      double* hist, void* stream)
{
    if (!c) return fail(nullptr, QCAMS_EINVAL, "null context");
    qcams_run_opts o;
    if (int rc = run_args(c, opts, st, sample, out, ids, xs, &o)) return rc;
    if (o.graph) return fail(c, QCAMS_EINVAL, "graph mode captures graphs: use qcams_run");
    if (c->n_total > kScratchItems)
        return fail(c, QCAMS_EINVAL, "%lld trajectories exceed the static scratch limit of %lld",
                    (long long)c->n_total, (long long)kScratchItems);
    if (c->n_xchunks > kScratchChunks)
        return fail(c, QCAMS_EINVAL, "%lld reduction chunks exceed the static scratch limit of %lld",
                    (long long)c->n_xchunks, (long long)kScratchChunks);
    unsigned char* base = scratch_of(c->device);
    if (!base) return fail(c, QCAMS_EINVAL, "no static scratch on device %d", c->device);
    HIP_OK(c, hipSetDevice(c->device));
    const RunBufs B{(unsigned long long*)base, (int64_t*)(base + kScratchOrderOff),
                    (double*)(base + kScratchPartOff)};
    hipStream_t s = (hipStream_t)stream;
    enqueue_pre(c, &o, B, st, sample, ids, s);
    if (enqueue_persistent(c, &o, B, st, s) != QCAMS_OK)
        return fail(c, QCAMS_EHIP, "run launch: %s", hipGetErrorString(hipGetLastError()));
    enqueue_post(c, B, st, out, ids, sample, xs, hist, s);
    HIP_OK(c, hipGetLastError());
    return QCAMS_OK;
}

// One timed run (minimum over reps) of option set `o`.
static int tune_time(qcams_ctx* c, const qcams_run_opts* o, const qcams_state* st,
                     const qcams_outcome* out, int64_t* ids, double* xs, int reps, hipStream_t s,
                     hipEvent_t e0, hipEvent_t e1, double* tmin)
{
    *tmin = 1e300;
    for (int r = 0; r < reps; ++r) {
        if (hipEventRecord(e0, s) != hipSuccess) return QCAMS_EHIP;
        int rc = qcams_run(c, o, st, nullptr, out, ids, xs, nullptr, s);
        if (rc != QCAMS_OK) return rc;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            return QCAMS_EHIP;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return QCAMS_EHIP;
        *tmin = fmin(*tmin, (double)ms);
    }
    return QCAMS_OK;
}

// Largest |H(t_f) - H(0)| / escale over the trajectories of the last run that
// did not fail (host copy of the outcome; the autotuner is synchronous).
static int tune_energy(qcams_ctx* c, const qcams_outcome* out, double* worst)
{
    const int64_t n = c->n_total;
    std::vector<double> dE((size_t)n);
    std::vector<uint8_t> lab((size_t)n);
    if (n > 0) {
        if (hipMemcpy(dE.data(), out->d + 3 * out->ld, n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(lab.data(), out->label, n, hipMemcpyDeviceToHost) != hipSuccess)
            return QCAMS_EHIP;
    }
    double w = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (lab[(size_t)i] != QCAMS_FAILED) w = fmax(w, fabs(dE[(size_t)i]));
    *worst = w;
    return QCAMS_OK;
}

// Autotune results of this process, keyed by what decides them: the device,
// the kernel specialisation, the variant search and its gate, the size of
// the installed work, and a hash of everything else a run depends on -- the
// system (masses, pair parameters and shapes), every integration parameter
// and the installed instance table (energies, levels, impact parameters,
// seeds, id ranges).  Two workloads of the same size but other content (which
// may keep a different RK variant inside the energy gate) get their own
// entries.
struct TuneKey {
    int device, kinds, lj126, search_rk;
    double gate;
    int64_t n_total;
    int32_t n_inst;
    uint64_t content;
    bool operator<(const TuneKey& o) const
    {
        return std::tie(device, kinds, lj126, search_rk, gate, n_total, n_inst, content) <
               std::tie(o.device, o.kinds, o.lj126, o.search_rk, o.gate, o.n_total, o.n_inst,
                        o.content);
    }
};

// FNV-1a over raw bytes (the hashed structures are value-initialised, so
// their padding is zero)
static uint64_t fnv1a(uint64_t h, const void* p, size_t n)
{
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

static uint64_t tune_content(const qcams_ctx* c)
{
    uint64_t h = 14695981039346656037ull;
    h = fnv1a(h, &c->sys, sizeof c->sys);
    h = fnv1a(h, &c->prm, sizeof c->prm);
    h = fnv1a(h, &c->level_method, sizeof c->level_method);
    if (!c->h_inst.empty()) h = fnv1a(h, c->h_inst.data(), c->h_inst.size() * sizeof(Inst));
    return h;
}
struct TuneVal {
    qcams_run_opts opts;
    double ms;
};
static std::mutex g_tune_mu;
static std::map<TuneKey, TuneVal> g_tune;

static int autotune_search(qcams_ctx* c, const qcams_state* st, const qcams_outcome* out,
                           int64_t* ids, double* xs, int32_t reps, int32_t search_rk,
                           double energy_gate, qcams_run_opts* best, double* best_ms);

int qcams_autotune(qcams_ctx* c, const qcams_state* st, const qcams_outcome* out, int64_t* ids,
                   double* xs, int32_t reps, int32_t search_rk, double energy_gate,
                   qcams_run_opts* best, double* best_ms)
{
    if (!c) return fail(nullptr, QCAMS_EINVAL, "null context");
    if (!best) return fail(c, QCAMS_EINVAL, "null result");
    if (search_rk != 0 && search_rk != 1) return fail(c, QCAMS_EINVAL, "search_rk must be 0 or 1");
    const TuneKey key{c->device, c->kinds, c->lj126 ? 1 : 0, search_rk,
                      search_rk ? energy_gate : 0.0, c->n_total, c->n_inst, tune_content(c)};
    if (reps >= 0) {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            *best = it->second.opts;
            if (best_ms) *best_ms = it->second.ms;
            return QCAMS_OK;
        }
    }
    double ms = 0.0;
    const int rc = autotune_search(c, st, out, ids, xs, reps < 0 ? -reps : (reps < 1 ? 1 : reps),
                                   search_rk, energy_gate, best, &ms);
    if (rc != QCAMS_OK) return rc;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune[key] = TuneVal{*best, ms};
    }
    if (best_ms) *best_ms = ms;
    return QCAMS_OK;
}

static int autotune_search(qcams_ctx* c, const qcams_state* st, const qcams_outcome* out,
                           int64_t* ids, double* xs, int32_t reps, int32_t search_rk,
                           double energy_gate, qcams_run_opts* best, double* best_ms)
{
    HIP_OK(c, hipSetDevice(c->device));
    hipStream_t s = nullptr;
    HIP_OK(c, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_OK(c, hipEventCreate(&e0));
    HIP_OK(c, hipEventCreate(&e1));
    double best_t = 1e300;
    qcams_run_opts bo{};
    int rc = QCAMS_OK;
    if (c->n_cu == 0) {
        int cu = 0;
        HIP_OK(c, hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, c->device));
        c->n_cu = cu > 0 ? cu : 256;
    }
    // Variant first (default schedule), among those that keep the energy gate;
    // then the schedule for the chosen variant.  The variant changes results
    // (a different integrator); the schedule does not.
    int rk = 0;
    if (search_rk) {
        double tv = 1e300;
        bool any = false;
        for (int v = 1; v <= 2 && rc == QCAMS_OK; ++v) {
            qcams_run_opts o{};
            o.refill_min = 1;
            o.check_every = 8;
            o.lpt = 1;
            o.rk = v;
            double t = 0.0, worst = 0.0;
            rc = tune_time(c, &o, st, out, ids, xs, reps, s, e0, e1, &t);
            if (rc == QCAMS_OK) rc = tune_energy(c, out, &worst);
            if (rc == QCAMS_OK && (energy_gate <= 0.0 || worst < energy_gate) && t < tv) {
                tv = t;
                rk = v;
                any = true;
            }
        }
        if (rc == QCAMS_OK && !any) rc = QCAMS_EINVAL;
    }
    // coordinate descent over the schedule options, two sweeps, from the
    // defaults: lanes per trajectory, grid, refill threshold, check interval,
    // instance order
    qcams_run_opts cur{};
    cur.blocks = c->n_cu;
    cur.refill_min = 1;
    cur.check_every = 8;
    cur.lpt = 1;
    cur.graph = 0;
    cur.rk = rk;
    cur.lanes = 4;
    if (rc == QCAMS_OK) rc = tune_time(c, &cur, st, out, ids, xs, reps, s, e0, e1, &best_t);
    bo = cur;
    const int nb = 4, nr = 3, nc = 3;
    const int blocks_c[nb] = {c->n_cu, 2 * c->n_cu, 3 * c->n_cu, 4 * c->n_cu};
    const int refill_c[nr] = {1, 4, 16};
    const int check_c[nc] = {1, 4, 8};
    for (int sweep = 0; sweep < 2 && rc == QCAMS_OK; ++sweep)
        for (int dim = 0; dim < 5 && rc == QCAMS_OK; ++dim) {
            const int nv = dim == 0 ? 3 : dim == 1 ? nb : dim == 2 ? nr : dim == 3 ? nc : 2;
            for (int v = 0; v < nv && rc == QCAMS_OK; ++v) {
                qcams_run_opts o = bo;
                if (dim == 0) o.lanes = v == 0 ? 4 : (v == 1 ? 1 : 8);
                else if (dim == 1) o.blocks = blocks_c[v];
                else if (dim == 2) o.refill_min = refill_c[v];
                else if (dim == 3) o.check_every = check_c[v];
                else o.lpt = 1 - v;
                if (o.lanes == bo.lanes && o.blocks == bo.blocks && o.refill_min == bo.refill_min &&
                    o.check_every == bo.check_every && o.lpt == bo.lpt)
                    continue;
                double tmin = 1e300;
                rc = tune_time(c, &o, st, out, ids, xs, reps, s, e0, e1, &tmin);
                if (rc == QCAMS_OK && tmin < best_t) {
                    best_t = tmin;
                    bo = o;
                }
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    if (rc == QCAMS_EINVAL) return fail(c, rc, "no RK variant keeps the energy gate");
    if (rc != QCAMS_OK) return rc == QCAMS_EHIP ? fail(c, rc, "autotune run failed") : rc;
    *best = bo;
    if (best_ms) *best_ms = best_t;
    return QCAMS_OK;
}

int qcams_grid_groups(qcams_ctx* c, int32_t* n_groups, int32_t* group_of)
{
    if (!c || !n_groups) return fail(c, QCAMS_EINVAL, "null argument");
    if (c->n_inst < 1) return fail(c, QCAMS_EINVAL, "no instances installed");
    *n_groups = c->n_groups;
    if (group_of)
        for (int k = 0; k < c->n_inst; ++k) group_of[k] = c->h_group_of[k];
    return QCAMS_OK;
}

int qcams_grid_cross_sections(qcams_ctx* c, const double* xs, double* out, void* stream)
{
    if (!c) return fail(nullptr, QCAMS_EINVAL, "null context");
    if (c->n_inst < 1) return fail(c, QCAMS_EINVAL, "no instances installed");
    if (c->n_groups == 0) return QCAMS_OK;
    if (!xs || !out) return fail(c, QCAMS_EINVAL, "null buffer");
    HIP_OK(c, hipSetDevice(c->device));
    hipLaunchKernelGGL(k_grid_xs, dim3(grid_of(c->n_groups, 64)), dim3(64), 0, (hipStream_t)stream,
                       c->d_inst, c->d_grid_inst, c->d_grid_off, c->n_groups, c->sys.mu123, xs, out);
    HIP_OK(c, hipGetLastError());
    return QCAMS_OK;
}

int qcams_last_run_options(qcams_ctx* c, qcams_run_opts* used)
{
    if (!c || !used) return fail(c, QCAMS_EINVAL, "null argument");
    if (!c->has_run) return fail(c, QCAMS_EINVAL, "no run recorded");
    *used = c->last_opts;
    return QCAMS_OK;
}

int qcams_last_run_wave_steps(qcams_ctx* c, int64_t* wave_steps)
{
    if (!c || !wave_steps) return fail(c, QCAMS_EINVAL, "null argument");
    if (!c->has_run || !c->last_counter) return fail(c, QCAMS_EINVAL, "no run recorded");
    HIP_OK(c, hipSetDevice(c->device));
    HIP_OK(c, hipEventSynchronize(c->ev_prop[1]));
    unsigned long long v = 0;
    HIP_OK(c, hipMemcpy(&v, c->last_counter + kWaveSteps, sizeof v, hipMemcpyDeviceToHost));
    *wave_steps = (int64_t)v;
    return QCAMS_OK;
}

int qcams_last_run_kernel_ms(qcams_ctx* c, double* ms)
{
    if (!c || !ms) return fail(c, QCAMS_EINVAL, "null argument");
    if (!c->ev_prop[0] || !c->ev_prop[1]) return fail(c, QCAMS_EINVAL, "no run recorded");
    HIP_OK(c, hipSetDevice(c->device));
    HIP_OK(c, hipEventSynchronize(c->ev_prop[1]));
    float f = 0.f;
    HIP_OK(c, hipEventElapsedTime(&f, c->ev_prop[0], c->ev_prop[1]));
    *ms = (double)f;
    return QCAMS_OK;
}


int qcams_mlp_features(qcams_ctx* c, const int64_t* ids, const double* sample, int64_t sample_ld,
                       const qcams_outcome* out, int64_t n, float* x, int32_t* y, void* stream)
{
    if (!c) return fail(nullptr, QCAMS_EINVAL, "null context");
    if (c->n_inst < 1) return fail(c, QCAMS_EINVAL, "no instances installed");
    if (n < 0 || (n > 0 && (!ids || !sample || !out || !out->label || !x || !y || sample_ld < n)))
        return fail(c, QCAMS_EINVAL, "bad arguments");
    if (n == 0) return QCAMS_OK;
    HIP_OK(c, hipSetDevice(c->device));
    hipLaunchKernelGGL(k_mlp_features, dim3(grid_of(n, 256)), dim3(256), 0, (hipStream_t)stream,
                       c->d_inst, c->n_inst, ids, sample, sample_ld, out->label, n, x, y);
    HIP_OK(c, hipGetLastError());
    return QCAMS_OK;
}

static int ensure_prop(qcams_ctx* c)
{
    if (c->d_prop_q) return QCAMS_OK;
    if (hipMalloc(&c->d_prop_q, kCells * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->d_prop_cdf, kCells * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->d_cell_x, kCells * 6 * sizeof(float)) != hipSuccess ||
        hipMalloc(&c->d_cell_p, kCells * 4 * sizeof(float)) != hipSuccess)
        return fail(c, QCAMS_ENOMEM, "proposal tables allocation failed");
    return QCAMS_OK;
}

int qcams_proposal_build(qcams_ctx* c, qcams_mlp* mlp, int32_t inst, int32_t channel, double alpha,
                         double* q)
{
    if (!c) return fail(nullptr, QCAMS_EINVAL, "null context");
    if (inst < 0 || inst >= c->n_inst || channel < 0 || channel > 3 || !(alpha > 0.0) || !(alpha <= 1.0) ||
        (!mlp && alpha < 1.0))
        return fail(c, QCAMS_EINVAL, "bad arguments");
    HIP_OK(c, hipSetDevice(c->device));
    if (int rc = ensure_prop(c)) return rc;
    const float* prob = nullptr;
    if (mlp && alpha < 1.0) {
        hipLaunchKernelGGL(k_cell_features, dim3(kCells / 256), dim3(256), 0, 0, c->d_inst, inst, c->d_cell_x);
        HIP_OK(c, hipGetLastError());
        const int rc = qcams_mlp_forward(mlp, c->d_cell_x, kCells, c->d_cell_p, nullptr);
        if (rc != QCAMS_OK) return fail(c, rc, "network forward: %s", qcams_mlp_last_error(mlp));
        prob = c->d_cell_p;
    }
    hipLaunchKernelGGL(k_prop_q, dim3(1), dim3(256), 0, 0, prob, channel, alpha, c->d_prop_q);
    hipLaunchKernelGGL(k_prop_cdf, dim3(1), dim3(256), 0, 0, c->d_prop_q, c->d_prop_cdf);
    HIP_OK(c, hipGetLastError());
    if (q) HIP_OK(c, hipMemcpy(q, c->d_prop_q, kCells * sizeof(double), hipMemcpyDeviceToDevice));
    HIP_OK(c, hipDeviceSynchronize());
    return QCAMS_OK;
}

int qcams_proposal_set(qcams_ctx* c, const double* q_host)
{
    if (!c) return fail(nullptr, QCAMS_EINVAL, "null context");
    if (!q_host) return fail(c, QCAMS_EINVAL, "null table");
    double tot = 0.0;
    for (int k = 0; k < kCells; ++k) {
        if (!(q_host[k] > 0.0) || !is_finite(q_host[k]))
            return fail(c, QCAMS_EINVAL, "cell %d: probability must be positive and finite", k);
        tot += q_host[k];
    }
    HIP_OK(c, hipSetDevice(c->device));
    if (int rc = ensure_prop(c)) return rc;
    HIP_OK(c, hipMemcpy(c->d_prop_q, q_host, kCells * sizeof(double), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_prop_cdf, dim3(1), dim3(256), 0, 0, c->d_prop_q, c->d_prop_cdf);
    HIP_OK(c, hipGetLastError());
    HIP_OK(c, hipDeviceSynchronize());
    return QCAMS_OK;
}

}  // extern "C"
