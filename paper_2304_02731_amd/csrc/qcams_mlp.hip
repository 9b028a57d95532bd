// qcams_mlp.hip -- learned importance-sampling proposal (gfx950).
//
// A 6 -> 128 -> 128 -> 128 -> 4 ReLU network maps a trajectory's initial
// conditions to the probabilities of its outcome class (quench, r1, r2,
// dissociation).  Forward and backward passes run on the BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation); master weights, gradients
// and the Adam state are FP32.  The trained network defines a proposal over
// cells of (b^2, chi, cos theta) from which the initial-condition kernel
// draws trajectories with exact importance weights, so every estimator of
// the method stays unbiased (cross sections Eq. (13), (18)).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <new>
#include <vector>

#include "../../include/qcams.h"

namespace {

constexpr int kIn = 6, kHid = 128, kOut = 4;
constexpr int kInP = 32;    // input padded to one MFMA k-block
constexpr int kOutP = 16;   // output padded to one MFMA n-tile
constexpr int kTile = 64;   // samples per workgroup (4 waves x 16 rows)
// flat parameter offsets (input-major W[i][o], then b[o])
constexpr int oW1 = 0, ob1 = oW1 + kIn * kHid;
constexpr int oW2 = ob1 + kHid, ob2 = oW2 + kHid * kHid;
constexpr int oW3 = ob2 + kHid, ob3 = oW3 + kHid * kHid;
constexpr int oW4 = ob3 + kHid, ob4 = oW4 + kHid * kOut;
constexpr int kNParam = ob4 + kOut;
static_assert(kNParam == QCAMS_MLP_NPARAM, "parameter count");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ inline __bf16 to_bf16(float f) { return (__bf16)f; }   // round to nearest even
__device__ inline float from_bf16(__bf16 h) { return (float)h; }

// One 16x16 output tile: C[i][j] += sum_k A[i][k] B[k][j] over K = 32 per call.
// Lane l supplies A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16]
// (e = 0..7) and receives C[4 (l / 16) + e][l % 16] (e = 0..3).
__device__ inline floatx4 mfma(const bf16x8& a, const bf16x8& b, const floatx4& c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

struct Weights {
    const float* theta;      // FP32 master [kNParam]
    const __bf16* w1f;       // [128][32]   forward layout: [out][in]
    const __bf16* w2f;       // [128][128]
    const __bf16* w3f;       // [128][128]
    const __bf16* w4f;       // [16][128]
    const __bf16* w2b;       // [128][128]  backward layout: [in][out]
    const __bf16* w3b;       // [128][128]
    const __bf16* w4b;       // [128][32]
};

// A fragment of a row-major bf16 matrix (leading dimension ld) at (r0, k0)
__device__ inline bf16x8 frag_rows(const __bf16* m, int ld, int r0, int k0, int lane)
{
    return *reinterpret_cast<const bf16x8*>(m + (r0 + (lane & 15)) * ld + k0 + 8 * (lane >> 4));
}

// A fragment of the transpose: element (r, k) = m[(k0 + k) * ld + r0 + r]
__device__ inline bf16x8 frag_cols(const __bf16* m, int ld, int r0, int k0, int lane)
{
    bf16x8 v;
    const int r = r0 + (lane & 15), k = k0 + 8 * (lane >> 4);
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = m[(k + e) * ld + r];
    return v;
}

// Dense layer on one wave's 16 rows: out[16][128] = act(in[16][K] W + b).
// in: LDS row-major [16][K]; wf: [128][K] (forward layout); out: LDS row-major.
template <int K, bool Relu>
__device__ inline void dense16(const __bf16* in, const __bf16* wf, const float* bias, __bf16* out,
                               float* zout, int lane)
{
#pragma unroll 1
    for (int t = 0; t < kHid / 16; ++t) {
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < K; kk += 32)
            acc = mfma(frag_rows(in, K, 0, kk, lane), frag_rows(wf, K, 16 * t, kk, lane), acc);
        const int j = 16 * t + (lane & 15);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = 4 * (lane >> 4) + e;
            float z = acc[e] + bias[j];
            if (zout) zout[i * kHid + j] = z;
            if (Relu) z = fmaxf(z, 0.f);
            out[i * kHid + j] = to_bf16(z);
        }
    }
}

// Forward of one wave's 16 samples up to the logits (written to lg[16][4]).
// x0: LDS [16][32] bf16 input rows; h1..h3: LDS [16][128] bf16.
__device__ inline void forward16(const Weights& W, const __bf16* x0, __bf16* h1, __bf16* h2,
                                 __bf16* h3, float* lg, int lane)
{
    dense16<kInP, true>(x0, W.w1f, W.theta + ob1, h1, nullptr, lane);
    __syncthreads();
    dense16<kHid, true>(h1, W.w2f, W.theta + ob2, h2, nullptr, lane);
    __syncthreads();
    dense16<kHid, true>(h2, W.w3f, W.theta + ob3, h3, nullptr, lane);
    __syncthreads();
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < kHid; kk += 32)
        acc = mfma(frag_rows(h3, kHid, 0, kk, lane), frag_rows(W.w4f, kHid, 0, kk, lane), acc);
    const int j = lane & 15;
    if (j < kOut) {
#pragma unroll
        for (int e = 0; e < 4; ++e) lg[(4 * (lane >> 4) + e) * kOut + j] = acc[e] + W.theta[ob4 + j];
    }
    __syncthreads();
}

// stage 16 input rows (6 features, zero padded to 32) as bf16
__device__ inline void load_x16(const float* x, const int32_t* idx, int64_t row0, int64_t n,
                                __bf16* x0, int lane)
{
    for (int q = lane; q < 16 * kInP; q += 64) {
        const int i = q / kInP, k = q % kInP;
        const int64_t r = row0 + i;
        float v = 0.f;
        if (r < n && k < kIn) v = x[(idx ? (int64_t)idx[r] : r) * kIn + k];
        x0[i * kInP + k] = to_bf16(v);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// inference: probabilities of the four classes
//
// Each workgroup copies the forward weights (bf16) and biases into LDS once
// and then walks groups of 128 rows (two 16-row tiles per wave) with a
// grid-stride loop, so every MFMA takes its weight fragment from LDS rather
// than from the cache.  LDS rows are padded by 8 bf16 (16 bytes): the 16 rows
// of a fragment then start in different banks.  The arithmetic is that of
// the training kernel's forward pass (the same MFMA sequence over k, bias,
// ReLU and bf16 rounding per layer).
// ---------------------------------------------------------------------------
constexpr int kLdIn = kInP + 8;    // padded LDS row strides (elements)
constexpr int kLdHid = kHid + 8;

// The lanes of one wave exchange rows through LDS: its LDS operations run
// in order, so it is enough that the compiler keeps them in order and that
// the stores have completed.
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Dense layer on one wave's 32 rows (two 16-row tiles) with LDS operands:
// out = act(in W + b), computed transposed (out^T = W^T in^T: the weight
// fragment is the MFMA's A operand, the rows' fragment its B operand), so
// that each lane receives four consecutive output features of one row and
// stores them with one 8-byte write.  All input fragments are read before
// the first output is written, so `out` may be `in` (in place); the two
// tiles' MFMA chains run side by side.
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
template <int K, bool Relu>
__device__ inline void dense32_lds(const __bf16* in, int ldi, const __bf16* wf, int ldw,
                                   const float* bias, __bf16* out, int ldo, int lane)
{
    constexpr int KB = K / 32;
    bf16x8 h[2][KB];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) h[r][kb] = frag_rows(in, ldi, 16 * r, 32 * kb, lane);
    floatx4 acc[2][kHid / 16];
#pragma unroll
    for (int t = 0; t < kHid / 16; ++t) {
        acc[0][t] = floatx4{0.f, 0.f, 0.f, 0.f};
        acc[1][t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            const bf16x8 w = frag_rows(wf, ldw, 16 * t, 32 * kb, lane);
            acc[0][t] = mfma(w, h[0][kb], acc[0][t]);
            acc[1][t] = mfma(w, h[1][kb], acc[1][t]);
        }
    }
    const int i0 = lane & 15, j0 = 4 * (lane >> 4);
#pragma unroll
    for (int t = 0; t < kHid / 16; ++t) {
        const floatx4 bj = *reinterpret_cast<const floatx4*>(bias + 16 * t + j0);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            bf16x4 o;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float z = acc[r][t][e] + bj[e];
                if (Relu) z = fmaxf(z, 0.f);
                o[e] = to_bf16(z);
            }
            *reinterpret_cast<bf16x4*>(out + (16 * r + i0) * ldo + 16 * t + j0) = o;
        }
    }
}

// rows x cols bf16 matrix (16-byte row chunks) from global into LDS with a
// padded row stride
__device__ inline void stage_rows(const __bf16* src, int rows, int cols, __bf16* dst, int ld, int tid)
{
    const int chunks = cols / 8;
    for (int q = tid; q < rows * chunks; q += 256) {
        const int r = q / chunks, c = q % chunks;
        *reinterpret_cast<bf16x8*>(dst + r * ld + 8 * c) =
            *reinterpret_cast<const bf16x8*>(src + r * cols + 8 * c);
    }
}

constexpr int kFwdRows = 32;               // rows per wave per iteration
constexpr int kFwdTile = 4 * kFwdRows;     // rows per workgroup per iteration

__global__ void __launch_bounds__(256) k_mlp_forward(Weights W, const float* x, int64_t n, float* prob)
{
    __shared__ __attribute__((aligned(16))) __bf16 s_w1[kHid * kLdIn];
    __shared__ __attribute__((aligned(16))) __bf16 s_w2[kHid * kLdHid];
    __shared__ __attribute__((aligned(16))) __bf16 s_w3[kHid * kLdHid];
    __shared__ __attribute__((aligned(16))) __bf16 s_w4[kOutP * kLdHid];
    __shared__ __attribute__((aligned(16))) float s_b[3 * kHid + kOut];
    __shared__ __attribute__((aligned(16))) __bf16 s_x[4][kFwdRows * kLdIn];
    __shared__ __attribute__((aligned(16))) __bf16 s_h[4][kFwdRows * kLdHid];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    stage_rows(W.w1f, kHid, kInP, s_w1, kLdIn, tid);
    stage_rows(W.w2f, kHid, kHid, s_w2, kLdHid, tid);
    stage_rows(W.w3f, kHid, kHid, s_w3, kLdHid, tid);
    stage_rows(W.w4f, kOutP, kHid, s_w4, kLdHid, tid);
    for (int q = tid; q < kHid; q += 256) {
        s_b[q] = W.theta[ob1 + q];
        s_b[kHid + q] = W.theta[ob2 + q];
        s_b[2 * kHid + q] = W.theta[ob3 + q];
    }
    if (tid < kOut) s_b[3 * kHid + tid] = W.theta[ob4 + tid];
    __syncthreads();
    const int64_t groups = (n + kFwdTile - 1) / kFwdTile;
    __bf16* xw = s_x[wave];
    __bf16* hw = s_h[wave];
    // each wave works on its own LDS rows: the waves need not wait for each other
    for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const int64_t row0 = g * kFwdTile + kFwdRows * wave;
        for (int q = lane; q < kFwdRows * kInP; q += 64) {
            const int i = q / kInP, k = q % kInP;
            const int64_t r = row0 + i;
            float v = 0.f;
            if (r < n && k < kIn) v = x[r * kIn + k];
            xw[i * kLdIn + k] = to_bf16(v);
        }
        wave_lds_sync();
        dense32_lds<kInP, true>(xw, kLdIn, s_w1, kLdIn, s_b, hw, kLdHid, lane);
        wave_lds_sync();
        dense32_lds<kHid, true>(hw, kLdHid, s_w2, kLdHid, s_b + kHid, hw, kLdHid, lane);
        wave_lds_sync();
        dense32_lds<kHid, true>(hw, kLdHid, s_w3, kLdHid, s_b + 2 * kHid, hw, kLdHid, lane);
        wave_lds_sync();
        // logits, transposed: lane l < 16 receives the four class logits of
        // row l of each tile; the softmax needs no exchange
        floatx4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int kk = 0; kk < kHid; kk += 32) {
            const bf16x8 w = frag_rows(s_w4, kLdHid, 0, kk, lane);
            acc[0] = mfma(w, frag_rows(hw, kLdHid, 0, kk, lane), acc[0]);
            acc[1] = mfma(w, frag_rows(hw, kLdHid, 16, kk, lane), acc[1]);
        }
        if (lane < 16) {
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int64_t row = row0 + 16 * r + lane;
                if (row < n) {
                    float z[kOut];
#pragma unroll
                    for (int c = 0; c < kOut; ++c) z[c] = acc[r][c] + s_b[3 * kHid + c];
                    const float m = fmaxf(fmaxf(z[0], z[1]), fmaxf(z[2], z[3]));
                    float e[kOut], sum = 0.f;
                    for (int c = 0; c < kOut; ++c) { e[c] = expf(z[c] - m); sum += e[c]; }
                    for (int c = 0; c < kOut; ++c) prob[row * kOut + c] = e[c] / sum;
                }
            }
        }
        wave_lds_sync();
    }
}

// ---------------------------------------------------------------------------
// gradient of the mean softmax cross-entropy over n rows (rows with label
// < 0 contribute nothing); one partial gradient per 64-row workgroup
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_mlp_grad(Weights W, const float* x, const int32_t* y, const int32_t* idx, int64_t n,
           float inv_n, float* partial, float* loss_part)
{
    __shared__ __attribute__((aligned(16))) __bf16 s_x[kTile * kInP];              // H0
    __shared__ __attribute__((aligned(16))) __bf16 s_h[3][kTile * kHid];           // H1..H3
    __shared__ __attribute__((aligned(16))) __bf16 s_dz[kTile * kHid];             // bf16 dZ of the current layer
    __shared__ float s_lg[kTile * kOut];
    __shared__ float s_red[256];
    __shared__ float s_colsum[4 * kHid];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, tid = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.x * kTile;
    float* P = partial + (int64_t)blockIdx.x * kNParam;
    // ---- forward (each wave: 16 rows), keeping the activations ----
    load_x16(x, idx, row0 + 16 * wave, n, s_x + 16 * wave * kInP, lane);
    forward16(W, s_x + 16 * wave * kInP, s_h[0] + 16 * wave * kHid, s_h[1] + 16 * wave * kHid,
              s_h[2] + 16 * wave * kHid, s_lg + 16 * wave * kOut, lane);
    __syncthreads();
    // ---- output layer: dZ4 = (p - onehot) / n ----
    float lsum = 0.f;
    if (tid < kTile) {
        const int64_t r = row0 + tid;
        const int lab = r < n ? y[idx ? (int64_t)idx[r] : r] : -1;
        float* z = s_lg + tid * kOut;
        if (lab >= 0 && lab < kOut) {
            const float m = fmaxf(fmaxf(z[0], z[1]), fmaxf(z[2], z[3]));
            float e[kOut], s = 0.f;
            for (int c = 0; c < kOut; ++c) { e[c] = expf(z[c] - m); s += e[c]; }
            for (int c = 0; c < kOut; ++c) z[c] = (e[c] / s - (c == lab ? 1.f : 0.f)) * inv_n;
            lsum = -logf(e[lab] / s);
        } else {
            for (int c = 0; c < kOut; ++c) z[c] = 0.f;
        }
    }
    s_red[tid] = lsum;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) s_red[tid] += s_red[tid + s];
        __syncthreads();
    }
    if (tid == 0) loss_part[blockIdx.x] = s_red[0];
    // db4 (FP32 dZ) and dW4 = H3^T bf16(dZ4)
    if (tid < kOut) {
        float s = 0.f;
        for (int r = 0; r < kTile; ++r) s += s_lg[r * kOut + tid];
        P[ob4 + tid] = s;
    }
    for (int q = tid; q < kHid * kOut; q += 256) {
        const int i = q / kOut, c = q % kOut;
        float s = 0.f;
        for (int r = 0; r < kTile; ++r)
            s += from_bf16(s_h[2][r * kHid + i]) * from_bf16(to_bf16(s_lg[r * kOut + c]));
        P[oW4 + i * kOut + c] = s;
    }
    // dH3 = bf16(dZ4) W4^T, dZ3 = dH3 * [H3 > 0]; column sums -> db3
    {
        const int j = tid & (kHid - 1), half = tid >> 7;
        float cs = 0.f;
        for (int r = half; r < kTile; r += 2) {
            float dh = 0.f;
            for (int c = 0; c < kOut; ++c)
                dh += from_bf16(to_bf16(s_lg[r * kOut + c])) * from_bf16(W.w4b[j * 32 + c]);
            const float dz = from_bf16(s_h[2][r * kHid + j]) > 0.f ? dh : 0.f;
            cs += dz;
            s_dz[r * kHid + j] = to_bf16(dz);
        }
        s_red[tid] = cs;
        __syncthreads();
        if (tid < kHid) P[ob3 + tid] = s_red[tid] + s_red[tid + kHid];
        __syncthreads();
    }
    // layers 3, 2, 1: dW = H^T bf16(dZ) (MFMA over the 64 rows), then dH = dZ W^T
    for (int layer = 3; layer >= 1; --layer) {
        const __bf16* Hin = layer == 1 ? s_x : s_h[layer - 2];
        const int kin = layer == 1 ? kInP : kHid;
        const int oW = layer == 3 ? oW3 : (layer == 2 ? oW2 : oW1);
        const int nin = layer == 1 ? kIn : kHid;
        // dW[i][j] = sum_r Hin[r][i] dZ[r][j]: tiles (i/16, j/16), K = 64 rows
        const int ntile_i = kin / 16, ntiles = ntile_i * (kHid / 16);
        for (int t = wave; t < ntiles; t += 4) {
            const int ti = t % ntile_i, tj = t / ntile_i;
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < kTile; kk += 32)
                acc = mfma(frag_cols(Hin, kin, 16 * ti, kk, lane), frag_cols(s_dz, kHid, 16 * tj, kk, lane), acc);
            const int j = 16 * tj + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = 16 * ti + 4 * (lane >> 4) + e;
                if (i < nin) P[oW + i * kHid + j] = acc[e];
            }
        }
        if (layer == 1) break;
        __syncthreads();
        // dH = bf16(dZ) W^T (MFMA, each wave its 16 rows), masked by the
        // previous activation; written as the next dZ (FP32 column sums
        // give the bias gradient)
        const __bf16* wb = layer == 3 ? W.w3b : W.w2b;
        const __bf16* Hprev = s_h[layer - 2];
        float dzv[kHid / 16][4];
        for (int t = 0; t < kHid / 16; ++t) {
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < kHid; kk += 32)
                acc = mfma(frag_rows(s_dz + 16 * wave * kHid, kHid, 0, kk, lane),
                           frag_rows(wb, kHid, 16 * t, kk, lane), acc);
            const int j = 16 * t + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = 16 * wave + 4 * (lane >> 4) + e;
                dzv[t][e] = from_bf16(Hprev[i * kHid + j]) > 0.f ? acc[e] : 0.f;
            }
        }
        __syncthreads();   // every wave has finished reading s_dz
        for (int t = 0; t < kHid / 16; ++t) {
            const int j = 16 * t + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = 16 * wave + 4 * (lane >> 4) + e;
                s_dz[i * kHid + j] = to_bf16(dzv[t][e]);
            }
        }
        // bias gradient: FP32 column sums of dZ, each wave over its 16 rows
        // (lanes l, l+16, l+32, l+48 share column 16 t + (l & 15)), then the
        // four waves in a fixed order
        const int ob = layer == 3 ? ob2 : ob1;
        for (int t = 0; t < kHid / 16; ++t) {
            float v = dzv[t][0] + dzv[t][1] + dzv[t][2] + dzv[t][3];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if ((lane >> 4) == 0) s_colsum[wave * kHid + 16 * t + (lane & 15)] = v;
        }
        __syncthreads();
        if (tid < kHid)
            P[ob + tid] = ((s_colsum[tid] + s_colsum[kHid + tid]) + s_colsum[2 * kHid + tid]) +
                          s_colsum[3 * kHid + tid];
        __syncthreads();
    }
}

// sum of the partial gradients in a fixed order, and the mean loss
__global__ void k_mlp_reduce(const float* partial, int nblk, float* grad, const float* loss_part,
                             float inv_n, float* loss)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kNParam) {
        float s = 0.f;
        for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * kNParam + p];
        grad[p] = s;
    }
    if (p == 0 && loss) {
        float s = 0.f;
        for (int b = 0; b < nblk; ++b) s += loss_part[b];
        loss[0] += s * inv_n;
    }
}

// bf16 copies of the weights in the forward ([out][in]) and backward
// ([in][out]) layouts, zero padded
__global__ void k_mlp_pack(const float* theta, __bf16* w1f, __bf16* w2f, __bf16* w3f, __bf16* w4f,
                           __bf16* w2b, __bf16* w3b, __bf16* w4b)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < kHid * kInP) {
        const int o = t / kInP, i = t % kInP;
        w1f[t] = to_bf16(i < kIn ? theta[oW1 + i * kHid + o] : 0.f);
    }
    if (t < kHid * kHid) {
        const int o = t / kHid, i = t % kHid;
        w2f[t] = to_bf16(theta[oW2 + i * kHid + o]);
        w3f[t] = to_bf16(theta[oW3 + i * kHid + o]);
        w2b[t] = to_bf16(theta[oW2 + t]);
        w3b[t] = to_bf16(theta[oW3 + t]);
    }
    if (t < kOutP * kHid) {
        const int o = t / kHid, i = t % kHid;
        w4f[t] = to_bf16(o < kOut ? theta[oW4 + i * kOut + o] : 0.f);
    }
    if (t < kHid * 32) {
        const int i = t / 32, o = t % 32;
        w4b[t] = to_bf16(o < kOut ? theta[oW4 + i * kOut + o] : 0.f);
    }
}

// Adam (Kingma & Ba 2015); the step counter lives on the device so that a
// captured epoch can be replayed
__global__ void k_mlp_adam(float* theta, float* m, float* v, const float* g, int* step, float lr,
                           float b1, float b2, float eps)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int t = *step + 1;
    if (p < kNParam) {
        const float gp = g[p];
        const float mp = b1 * m[p] + (1.f - b1) * gp;
        const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
        m[p] = mp;
        v[p] = vp;
        const float mh = mp / (1.f - powf(b1, (float)t));
        const float vh = vp / (1.f - powf(b2, (float)t));
        theta[p] -= lr * mh / (sqrtf(vh) + eps);
    }
}

__global__ void k_mlp_step_inc(int* step) { *step += 1; }
__global__ void k_zero1(float* p) { *p = 0.f; }

// He-uniform initialisation from a counter-based hash (weights), zero biases
__global__ void k_mlp_init(float* theta, uint64_t seed)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNParam) return;
    int fan_in;
    bool bias;
    if (p < ob1) { fan_in = kIn; bias = false; }
    else if (p < oW2) { fan_in = kIn; bias = true; }
    else if (p < ob2) { fan_in = kHid; bias = false; }
    else if (p < oW3) { fan_in = kHid; bias = true; }
    else if (p < ob3) { fan_in = kHid; bias = false; }
    else if (p < oW4) { fan_in = kHid; bias = true; }
    else if (p < ob4) { fan_in = kHid; bias = false; }
    else { fan_in = kHid; bias = true; }
    if (bias) { theta[p] = 0.f; return; }
    // splitmix64 of (seed, p)
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(p + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const double u = (double)(z >> 11) * 0x1.0p-53;
    theta[p] = (float)((2.0 * u - 1.0) * sqrt(6.0 / fan_in));
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct qcams_mlp {
    int device = 0;
    int n_cu = 256;   // compute units of the device (forward grid)
    float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    float* partial = nullptr;
    float* loss_part = nullptr;
    int64_t part_cap = 0;
    int* step = nullptr;
    __bf16 *w1f = nullptr, *w2f = nullptr, *w3f = nullptr, *w4f = nullptr;
    __bf16 *w2b = nullptr, *w3b = nullptr, *w4b = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t key[8] = {0};
    char err[512] = {0};
};

static char g_mlp_err[512];

static int mfail(qcams_mlp* m, int code, const char* fmt, ...)
{
    char* dst = m ? m->err : g_mlp_err;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(dst, 512, fmt, ap);
    va_end(ap);
    return code;
}

#define MHIP(m, expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return mfail(m, QCAMS_EHIP, "%s: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

static Weights weights_of(const qcams_mlp* m)
{
    return Weights{m->theta, m->w1f, m->w2f, m->w3f, m->w4f, m->w2b, m->w3b, m->w4b};
}

static void enqueue_pack(qcams_mlp* m, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_pack, dim3((kHid * kHid + 255) / 256), dim3(256), 0, s, m->theta, m->w1f,
                       m->w2f, m->w3f, m->w4f, m->w2b, m->w3b, m->w4b);
}

static int ensure_partial(qcams_mlp* m, int64_t nblk)
{
    if (nblk <= m->part_cap) return QCAMS_OK;
    if (m->partial) MHIP(m, hipFree(m->partial));
    if (m->loss_part) MHIP(m, hipFree(m->loss_part));
    m->partial = nullptr;
    m->loss_part = nullptr;
    m->part_cap = 0;
    if (hipMalloc(&m->partial, (size_t)nblk * kNParam * sizeof(float)) != hipSuccess ||
        hipMalloc(&m->loss_part, (size_t)nblk * sizeof(float)) != hipSuccess)
        return mfail(m, QCAMS_ENOMEM, "gradient partials allocation failed");
    m->part_cap = nblk;
    m->key[0] = 0;
    return QCAMS_OK;
}

static void enqueue_grad(qcams_mlp* m, const float* x, const int32_t* y, const int32_t* idx, int64_t n,
                         float* grad, float* loss, hipStream_t s)
{
    const int nblk = (int)((n + kTile - 1) / kTile);
    const float inv_n = 1.0f / (float)n;
    hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(256), 0, s, weights_of(m), x, y, idx, n, inv_n,
                       m->partial, m->loss_part);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kNParam + 255) / 256), dim3(256), 0, s, m->partial, nblk,
                       grad, m->loss_part, inv_n, loss);
}

extern "C" {

int qcams_mlp_create(qcams_mlp** out, int device, const float* params, uint64_t seed)
{
    if (!out) return mfail(nullptr, QCAMS_EINVAL, "null argument");
    *out = nullptr;
    qcams_mlp* m = new (std::nothrow) qcams_mlp();
    if (!m) return mfail(nullptr, QCAMS_ENOMEM, "host allocation failed");
    m->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete m;
        return mfail(nullptr, QCAMS_EHIP, "hipSetDevice failed");
    }
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cu > 0)
        m->n_cu = cu;
    bool ok = hipMalloc(&m->theta, kNParam * sizeof(float)) == hipSuccess &&
              hipMalloc(&m->m, kNParam * sizeof(float)) == hipSuccess &&
              hipMalloc(&m->v, kNParam * sizeof(float)) == hipSuccess &&
              hipMalloc(&m->grad, kNParam * sizeof(float)) == hipSuccess &&
              hipMalloc(&m->step, sizeof(int)) == hipSuccess &&
              hipMalloc(&m->w1f, kHid * kInP * sizeof(__bf16)) == hipSuccess &&
              hipMalloc(&m->w2f, kHid * kHid * sizeof(__bf16)) == hipSuccess &&
              hipMalloc(&m->w3f, kHid * kHid * sizeof(__bf16)) == hipSuccess &&
              hipMalloc(&m->w4f, kOutP * kHid * sizeof(__bf16)) == hipSuccess &&
              hipMalloc(&m->w2b, kHid * kHid * sizeof(__bf16)) == hipSuccess &&
              hipMalloc(&m->w3b, kHid * kHid * sizeof(__bf16)) == hipSuccess &&
              hipMalloc(&m->w4b, kHid * 32 * sizeof(__bf16)) == hipSuccess;
    if (!ok) {
        qcams_mlp_destroy(m);
        return mfail(nullptr, QCAMS_ENOMEM, "device allocation failed");
    }
    hipError_t e = hipMemset(m->m, 0, kNParam * sizeof(float));
    if (e == hipSuccess) e = hipMemset(m->v, 0, kNParam * sizeof(float));
    if (e == hipSuccess) e = hipMemset(m->step, 0, sizeof(int));
    if (e == hipSuccess) {
        if (params) e = hipMemcpy(m->theta, params, kNParam * sizeof(float), hipMemcpyHostToDevice);
        else hipLaunchKernelGGL(k_mlp_init, dim3((kNParam + 255) / 256), dim3(256), 0, 0, m->theta, seed);
    }
    if (e == hipSuccess) {
        enqueue_pack(m, 0);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        qcams_mlp_destroy(m);
        return mfail(nullptr, QCAMS_EHIP, "initialisation: %s", hipGetErrorString(e));
    }
    *out = m;
    return QCAMS_OK;
}

void qcams_mlp_destroy(qcams_mlp* m)
{
    if (!m) return;
    (void)hipSetDevice(m->device);
    if (m->exec) (void)hipGraphExecDestroy(m->exec);
    if (m->graph) (void)hipGraphDestroy(m->graph);
    if (m->cap) (void)hipStreamDestroy(m->cap);
    for (void* p : {(void*)m->theta, (void*)m->m, (void*)m->v, (void*)m->grad, (void*)m->partial,
                    (void*)m->loss_part, (void*)m->step, (void*)m->w1f, (void*)m->w2f, (void*)m->w3f,
                    (void*)m->w4f, (void*)m->w2b, (void*)m->w3b, (void*)m->w4b})
        if (p) (void)hipFree(p);
    delete m;
}

const char* qcams_mlp_last_error(const qcams_mlp* m) { return m ? m->err : g_mlp_err; }

int qcams_mlp_get_params(qcams_mlp* m, float* params)
{
    if (!m || !params) return mfail(m, QCAMS_EINVAL, "null argument");
    MHIP(m, hipSetDevice(m->device));
    MHIP(m, hipDeviceSynchronize());
    MHIP(m, hipMemcpy(params, m->theta, kNParam * sizeof(float), hipMemcpyDeviceToHost));
    return QCAMS_OK;
}

int qcams_mlp_set_params(qcams_mlp* m, const float* params)
{
    if (!m || !params) return mfail(m, QCAMS_EINVAL, "null argument");
    MHIP(m, hipSetDevice(m->device));
    MHIP(m, hipDeviceSynchronize());
    MHIP(m, hipMemcpy(m->theta, params, kNParam * sizeof(float), hipMemcpyHostToDevice));
    MHIP(m, hipMemset(m->m, 0, kNParam * sizeof(float)));
    MHIP(m, hipMemset(m->v, 0, kNParam * sizeof(float)));
    MHIP(m, hipMemset(m->step, 0, sizeof(int)));
    enqueue_pack(m, 0);
    MHIP(m, hipGetLastError());
    MHIP(m, hipDeviceSynchronize());
    return QCAMS_OK;
}

int qcams_mlp_forward(qcams_mlp* m, const float* x, int64_t n, float* prob, void* stream)
{
    if (!m || n < 0 || (n > 0 && (!x || !prob))) return mfail(m, QCAMS_EINVAL, "bad arguments");
    if (n == 0) return QCAMS_OK;
    MHIP(m, hipSetDevice(m->device));
    // one resident workgroup per CU (the LDS copy of the weights): as many
    // workgroups as CUs, or fewer for small n
    const int64_t groups = (n + kFwdTile - 1) / kFwdTile;
    const int64_t grid = groups < m->n_cu ? groups : m->n_cu;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream,
                       weights_of(m), x, n, prob);
    MHIP(m, hipGetLastError());
    return QCAMS_OK;
}

int qcams_mlp_gradient(qcams_mlp* m, const float* x, const int32_t* y, const int32_t* idx, int64_t n,
                       float* grad, float* loss, void* stream)
{
    if (!m || n < 1 || !x || !y || !grad) return mfail(m, QCAMS_EINVAL, "bad arguments");
    MHIP(m, hipSetDevice(m->device));
    if (int rc = ensure_partial(m, (n + kTile - 1) / kTile)) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (loss) hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, s, loss);
    enqueue_grad(m, x, y, idx, n, grad, loss, s);
    MHIP(m, hipGetLastError());
    return QCAMS_OK;
}

int qcams_mlp_train_epoch(qcams_mlp* m, const float* x, const int32_t* y, const int32_t* perm,
                          int64_t n, int32_t batch, float lr, float* loss_sum, void* stream)
{
    if (!m || !x || !y || !perm || !loss_sum || n < 1 || batch < 1 || !(lr > 0.f))
        return mfail(m, QCAMS_EINVAL, "bad arguments");
    MHIP(m, hipSetDevice(m->device));
    if (int rc = ensure_partial(m, (batch + kTile - 1) / kTile)) return rc;
    const int64_t nb = n / batch;   // full batches only
    if (nb < 1) return mfail(m, QCAMS_EINVAL, "fewer rows than one batch");
    const uint64_t key[8] = {1, (uint64_t)x, (uint64_t)y, (uint64_t)perm, (uint64_t)n,
                             (uint64_t)batch, (uint64_t)__builtin_bit_cast(uint32_t, lr),
                             (uint64_t)loss_sum};
    if (memcmp(key, m->key, sizeof key) != 0) {
        if (m->exec) { MHIP(m, hipGraphExecDestroy(m->exec)); m->exec = nullptr; }
        if (m->graph) { MHIP(m, hipGraphDestroy(m->graph)); m->graph = nullptr; }
        if (!m->cap) MHIP(m, hipStreamCreateWithFlags(&m->cap, hipStreamNonBlocking));
        MHIP(m, hipStreamBeginCapture(m->cap, hipStreamCaptureModeThreadLocal));
        hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, m->cap, loss_sum);
        for (int64_t b = 0; b < nb; ++b) {
            enqueue_grad(m, x, y, perm + b * batch, batch, m->grad, loss_sum, m->cap);
            hipLaunchKernelGGL(k_mlp_adam, dim3((kNParam + 255) / 256), dim3(256), 0, m->cap, m->theta,
                               m->m, m->v, m->grad, m->step, lr, 0.9f, 0.999f, 1e-8f);
            hipLaunchKernelGGL(k_mlp_step_inc, dim3(1), dim3(1), 0, m->cap, m->step);
            enqueue_pack(m, m->cap);
        }
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(m->cap, &g);
        if (e != hipSuccess) return mfail(m, QCAMS_EHIP, "capture: %s", hipGetErrorString(e));
        m->graph = g;
        MHIP(m, hipGraphInstantiate(&m->exec, g, nullptr, nullptr, 0));
        memcpy(m->key, key, sizeof key);
    }
    MHIP(m, hipGraphLaunch(m->exec, (hipStream_t)stream));
    return QCAMS_OK;
}

int qcams_mlp_adam(qcams_mlp* m, const float* grad, float lr, void* stream)
{
    if (!m || !grad || !(lr > 0.f)) return mfail(m, QCAMS_EINVAL, "bad arguments");
    MHIP(m, hipSetDevice(m->device));
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mlp_adam, dim3((kNParam + 255) / 256), dim3(256), 0, s, m->theta, m->m, m->v,
                       grad, m->step, lr, 0.9f, 0.999f, 1e-8f);
    hipLaunchKernelGGL(k_mlp_step_inc, dim3(1), dim3(1), 0, s, m->step);
    enqueue_pack(m, s);
    MHIP(m, hipGetLastError());
    return QCAMS_OK;
}

}  // extern "C"
