// qcams_dvr.hip -- internal energies of the molecule by the Colbert-Miller
// discrete variable representation (DVR), the paper's method for E(v, j)
// (Koots & Perez-Rios, arXiv:2304.02731, Sec. 2.1; grid keys npts, xmin,
// xmax of Sec. 3.1).
//
// READING: the particle-in-a-box DVR of Colbert and Miller on (a, b) =
// (xmin, xmax) with N = npts + 1 intervals and the npts interior points
// r_i = a + i (b - a) / N.  With L = b - a the kinetic matrix is
//   T_ii  = pi^2/(4 mu L^2) [(2N^2 + 1)/3 - 1/sin^2(pi i/N)],
//   T_ii' = pi^2/(4 mu L^2) (-1)^(i-i') [1/sin^2(pi (i-i')/(2N)) - 1/sin^2(pi (i+i')/(2N))],
// and V(r_i) + j(j+1)/(2 mu r_i^2) is added on the diagonal.
//
// The dense symmetric matrices (one per distinct j) are reduced to
// tridiagonal form by Householder reflections, A <- H A H with
// H = I - 2 v v^T, |v| = 1 (per column: the reflector, p = A v over the
// trailing block, q = 2 p - 2 (v.p) v, A <- A - v q^T - q v^T), then the
// lowest eigenvalues of the tridiagonal matrix are found by bisection on its
// Sturm sequence (the count of negative pivots of T - x I).  Both steps are
// backward stable; the matrices stay in device memory throughout.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "qcams_device.h"

using namespace qd;

namespace {

constexpr int kT = 256;

__global__ void k_dvr_build(Pot P, double mu, double a, double b, int n, const int* js, double* A)
{
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;
    const int m = blockIdx.z;
    if (col >= n || row >= n) return;
    const int N = n + 1;
    const double L = b - a;
    const double pref = kPi * kPi / (4.0 * mu * L * L);
    const int i = row + 1, k = col + 1;
    double t;
    if (i == k) {
        const double s = sin(kPi * i / N);
        t = pref * ((2.0 * N * N + 1.0) / 3.0 - 1.0 / (s * s));
        const double r = a + i * L / N;
        const double J2 = (double)js[m] * (js[m] + 1.0);
        t += pot_V(P, r) + J2 / (2.0 * mu * r * r);
    } else {
        const double s1 = sin(kPi * (i - k) / (2.0 * N)), s2 = sin(kPi * (i + k) / (2.0 * N));
        t = pref * (((i - k) & 1) ? -1.0 : 1.0) * (1.0 / (s1 * s1) - 1.0 / (s2 * s2));
    }
    A[((size_t)m * n + row) * n + col] = t;
}

// block sum of one value per thread; every thread gets the total
__device__ double block_total(double x, double* red)
{
    red[threadIdx.x] = x;
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double t = red[0];
    __syncthreads();
    return t;
}

// Reflector for column k of matrix m: v over rows k+1..n-1 (zero elsewhere),
// d[k] = A[k][k], e[k] = the new sub-diagonal entry.  One block per matrix.
__global__ void __launch_bounds__(kT) k_hh_vector(double* A, int n, int k, double* V, double* d,
                                                  double* e)
{
    __shared__ double red[kT];
    const int m = blockIdx.x;
    double* a = A + (size_t)m * n * n;
    double* v = V + (size_t)m * n;
    const double* rowk = a + (size_t)k * n;   // row k = column k (symmetric)
    double s = 0.0;
    for (int i = k + 2 + threadIdx.x; i < n; i += kT) s += rowk[i] * rowk[i];
    const double tail = block_total(s, red);   // |x|^2 without its first entry
    const double x0 = rowk[k + 1];
    const double sig = tail + x0 * x0;
    const bool refl = tail > 0.0;
    const double alpha = refl ? (x0 > 0.0 ? -sqrt(sig) : sqrt(sig)) : x0;
    // v = (x - alpha e1) / |x - alpha e1|,  |x - alpha e1|^2 = 2 (sig - alpha x0)
    const double inv = refl ? 1.0 / sqrt(2.0 * (sig - alpha * x0)) : 0.0;
    for (int i = threadIdx.x; i < n; i += kT) {
        double vi = 0.0;
        if (refl && i > k) vi = (i == k + 1 ? x0 - alpha : rowk[i]) * inv;
        v[i] = vi;
    }
    if (threadIdx.x == 0) {
        d[(size_t)m * n + k] = rowk[k];
        e[(size_t)m * n + k] = alpha;
    }
}

// p_i = sum_{j > k} A[j][i] v_j for i > k (A symmetric; reading column i
// along j keeps a wave's loads contiguous).
__global__ void __launch_bounds__(kT) k_hh_matvec(const double* A, int n, int k, const double* V,
                                                  double* Pv)
{
    const int m = blockIdx.y;
    const int i = k + 1 + blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const double* a = A + (size_t)m * n * n;
    const double* v = V + (size_t)m * n;
    double s = 0.0;
    for (int j = k + 1; j < n; ++j) s = fma(a[(size_t)j * n + i], v[j], s);
    Pv[(size_t)m * n + i] = s;
}

// q = 2 p - 2 (v.p) v over i > k, in place of p.  One block per matrix.
__global__ void __launch_bounds__(kT) k_hh_q(int n, int k, const double* V, double* Pv)
{
    __shared__ double red[kT];
    const int m = blockIdx.x;
    const double* v = V + (size_t)m * n;
    double* p = Pv + (size_t)m * n;
    double s = 0.0;
    for (int i = k + 1 + threadIdx.x; i < n; i += kT) s = fma(v[i], p[i], s);
    const double K = block_total(s, red);
    for (int i = k + 1 + threadIdx.x; i < n; i += kT) p[i] = 2.0 * p[i] - 2.0 * K * v[i];
}

// A <- A - v q^T - q v^T on the trailing block (rows and columns > k).
__global__ void __launch_bounds__(kT) k_hh_update(double* A, int n, int k, const double* V,
                                                  const double* Q)
{
    const int m = blockIdx.z;
    const int col = k + 1 + blockIdx.x * kT + threadIdx.x;
    const int row = k + 1 + blockIdx.y;
    if (col >= n || row >= n) return;
    const double* v = V + (size_t)m * n;
    const double* q = Q + (size_t)m * n;
    double& x = A[((size_t)m * n + row) * n + col];
    x = x - v[row] * q[col] - q[row] * v[col];
}

// number of eigenvalues of the tridiagonal (d, e) below x (Sturm count)
__device__ int sturm_below(const double* d, const double* e, int n, double x)
{
    int c = 0;
    double q = d[0] - x;
    if (q < 0.0) ++c;
    for (int i = 1; i < n; ++i) {
        if (q == 0.0) q = -1e-300;
        q = (d[i] - x) - e[i - 1] * e[i - 1] / q;
        if (q < 0.0) ++c;
    }
    return c;
}

// eigenvalue number r (0 = lowest) of each tridiagonal, by bisection
__global__ void k_tridiag_eig(const double* D, const double* E, int n, int K, double* out)
{
    const int m = blockIdx.y;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= K) return;
    const double* d = D + (size_t)m * n;
    const double* e = E + (size_t)m * n;
    double lo = d[0], hi = d[0];
    for (int i = 0; i < n; ++i) {   // Gershgorin bounds
        const double rad = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i < n - 1 ? fabs(e[i]) : 0.0);
        lo = fmin(lo, d[i] - rad);
        hi = fmax(hi, d[i] + rad);
    }
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        if (sturm_below(d, e, n, mid) > r) hi = mid;
        else lo = mid;
    }
    out[(size_t)m * K + r] = 0.5 * (lo + hi);
}

}  // namespace

// Lowest K eigenvalues of the DVR Hamiltonian of pair P for each of the nj
// values js (host), into out (host [nj][K]).  Returns 0, or -1 (bad
// arguments / allocation) / -2 (HIP error) with a message in err.  Internal
// to the library (C linkage, called by the API translation unit).
extern "C" int qd_dvr_eigenvalues(int device, const Pot& P, double mu, double a, double b, int n, int nj,
                       const int* js, int K, double* out, char* err, size_t errlen)
{
    if (n < 4 || nj < 1 || K < 1 || K > n || !(b > a) || !(a > 0.0)) {
        snprintf(err, errlen, "DVR: invalid grid or counts");
        return -1;
    }
    if (hipSetDevice(device) != hipSuccess) return -2;
    double *A = nullptr, *V = nullptr, *Pv = nullptr, *D = nullptr, *Ev = nullptr, *O = nullptr;
    int* dj = nullptr;
    const size_t nn = (size_t)n * n * nj;
    int rc = 0;
    if (hipMalloc(&A, nn * sizeof(double)) != hipSuccess ||
        hipMalloc(&V, (size_t)n * nj * sizeof(double)) != hipSuccess ||
        hipMalloc(&Pv, (size_t)n * nj * sizeof(double)) != hipSuccess ||
        hipMalloc(&D, (size_t)n * nj * sizeof(double)) != hipSuccess ||
        hipMalloc(&Ev, (size_t)n * nj * sizeof(double)) != hipSuccess ||
        hipMalloc(&O, (size_t)K * nj * sizeof(double)) != hipSuccess ||
        hipMalloc(&dj, nj * sizeof(int)) != hipSuccess) {
        snprintf(err, errlen, "DVR: device allocation failed");
        rc = -1;
    }
    if (rc == 0 && hipMemcpy(dj, js, nj * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) rc = -2;
    if (rc == 0) {
        hipLaunchKernelGGL(k_dvr_build, dim3((n + kT - 1) / kT, n, nj), dim3(kT), 0, 0, P, mu, a, b,
                           n, (const int*)dj, A);
        for (int k = 0; k + 2 < n; ++k) {
            const int mrem = n - k - 1;
            hipLaunchKernelGGL(k_hh_vector, dim3(nj), dim3(kT), 0, 0, A, n, k, V, D, Ev);
            hipLaunchKernelGGL(k_hh_matvec, dim3((mrem + kT - 1) / kT, nj), dim3(kT), 0, 0,
                               (const double*)A, n, k, (const double*)V, Pv);
            hipLaunchKernelGGL(k_hh_q, dim3(nj), dim3(kT), 0, 0, n, k, (const double*)V, Pv);
            hipLaunchKernelGGL(k_hh_update, dim3((mrem + kT - 1) / kT, mrem, nj), dim3(kT), 0, 0, A,
                               n, k, (const double*)V, (const double*)Pv);
        }
        if (hipGetLastError() != hipSuccess) rc = -2;
    }
    if (rc == 0) {
        // the last 2 x 2 block: d[n-2], d[n-1], e[n-2]
        std::vector<double> tail(3 * nj);
        for (int m = 0; m < nj && rc == 0; ++m) {
            const double* am = A + (size_t)m * n * n;
            double t[3];
            if (hipMemcpy(&t[0], am + (size_t)(n - 2) * n + (n - 2), sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
                hipMemcpy(&t[1], am + (size_t)(n - 1) * n + (n - 1), sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
                hipMemcpy(&t[2], am + (size_t)(n - 1) * n + (n - 2), sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
                hipMemcpy(D + (size_t)m * n + (n - 2), &t[0], 2 * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(Ev + (size_t)m * n + (n - 2), &t[2], sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
                rc = -2;
        }
    }
    if (rc == 0) {
        hipLaunchKernelGGL(k_tridiag_eig, dim3((K + 63) / 64, nj), dim3(64), 0, 0, (const double*)D,
                           (const double*)Ev, n, K, O);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpy(out, O, (size_t)K * nj * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
            rc = -2;
    }
    if (rc == -2) snprintf(err, errlen, "DVR: %s", hipGetErrorString(hipGetLastError()));
    for (void* q : {(void*)A, (void*)V, (void*)Pv, (void*)D, (void*)Ev, (void*)O, (void*)dj})
        if (q) (void)hipFree(q);
    return rc;
}
