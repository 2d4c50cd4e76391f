// Observable epilogue (Sec. 2), azimuthal average (eq. iqazi) and correlation
// functions (eqs. crrad, prrad) on gfx950.  All three are memory-bound and tiny
// next to the Fourier sums; they are written for determinism (fixed reduction
// orders, no floating-point atomics).
//
// Every cross section is a Hermitian form in the sums, so the epilogue works
// on the 4x4 spectral matrix G_ab = A_a conj(A_b) (formed on the fly from one
// amplitude set, or read as accumulated over objects/rotations).  With
// qhat = (0, sin t, cos t), Pp = I - qhat qhat^T and Q = qhat x (qhat x M) = -Pp M:
//   |Q|^2        = tr(H),                 H = Pp G_MM Pp
//   |Phat.Q|^2   = Phat^T H Phat
//   NM form      = -2 sum_a u_a Re G_{N,a},   u = Pp Phat
//   chiral term  = 2 [Px Im H_yz + Py Im H_zx + Pz Im H_xy]
// (the last from -i Phat.(Q x Q*) with Q_b conj(Q_c) = H_bc).
#include "numag_internal.h"
#include "phasor.h"

namespace numag {

struct C {
    double re, im;
};

__device__ __forceinline__ C cmk(double r, double i) { return C{r, i}; }
__device__ __forceinline__ C cconj(C a) { return C{a.re, -a.im}; }
__device__ __forceinline__ C cadd(C a, C b) { return C{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ C cscale(double s, C a) { return C{s * a.re, s * a.im}; }


// ---------------------------------------------------------------------------
// cross sections
// ---------------------------------------------------------------------------
__global__ void cross_section_kernel(Detector d, int64_t n_sets, const double *__restrict__ amp,
                                     const double *__restrict__ spec, numag_consts k, uint32_t mask,
                                     int n_out, double *__restrict__ out)
{
    const int64_t P = (int64_t)d.n0 * d.n1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_sets * P) return;
    const int64_t set = idx / P, p = idx % P;

    // spectral matrix G (complex 4x4, Hermitian)
    C G[4][4];
    if (amp != nullptr) {
        const double *a = amp + idx * 8;
        C A[4];
        for (int v = 0; v < 4; ++v) A[v] = cmk(a[2 * v], a[2 * v + 1]);
        for (int x = 0; x < 4; ++x)
            for (int y = 0; y < 4; ++y)
                G[x][y] = cmk(A[x].re * A[y].re + A[x].im * A[y].im, A[x].im * A[y].re - A[x].re * A[y].im);
    } else {
        const double *g = spec + idx * 16;
        const int pa[6] = {0, 0, 0, 1, 1, 2};
        const int pb[6] = {1, 2, 3, 2, 3, 3};
        for (int x = 0; x < 4; ++x) G[x][x] = cmk(g[x], 0.0);
        for (int tt = 0; tt < 6; ++tt) {
            C v = cmk(g[4 + 2 * tt], g[5 + 2 * tt]);
            G[pa[tt]][pb[tt]] = v;
            G[pb[tt]][pa[tt]] = cconj(v);
        }
    }

    double s, c;
    pixel_qhat(d, p, s, c);
    const double qh[3] = {0.0, s, c};
    double Pp[3][3];
    for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y) Pp[x][y] = (x == y ? 1.0 : 0.0) - qh[x] * qh[y];

    // H = Pp G_MM Pp
    C T[3][3], H[3][3];
    for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y) {
            C acc = cmk(0.0, 0.0);
            for (int z = 0; z < 3; ++z) acc = cadd(acc, cscale(Pp[x][z], G[1 + z][1 + y]));
            T[x][y] = acc;
        }
    for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y) {
            C acc = cmk(0.0, 0.0);
            for (int z = 0; z < 3; ++z) acc = cadd(acc, cscale(Pp[z][y], T[x][z]));
            H[x][y] = acc;
        }
    const double Ph[3] = {k.P[0], k.P[1], k.P[2]};
    double u[3];
    for (int x = 0; x < 3; ++x) u[x] = Pp[x][0] * Ph[0] + Pp[x][1] * Ph[1] + Pp[x][2] * Ph[2];

    const double cf = k.scale / k.V;
    const double b2 = k.bH * k.bH;
    const double absQ2 = H[0][0].re + H[1][1].re + H[2][2].re;
    double pq2 = 0.0;
    for (int x = 0; x < 3; ++x)
        for (int y = 0; y < 3; ++y) pq2 += Ph[x] * Ph[y] * H[x][y].re;
    double nmf = 0.0;
    for (int x = 0; x < 3; ++x) nmf += -2.0 * u[x] * G[0][1 + x].re;
    const double chif = 2.0 * (Ph[0] * H[1][2].im + Ph[1] * H[2][0].im + Ph[2] * H[0][1].im);

    double obs[13];
    const double N = cf * G[0][0].re;
    const double M = cf * b2 * absQ2;
    const double NM = cf * k.bH * nmf;
    const double Pv = cf * b2 * pq2;
    const double CHI = cf * b2 * chif;
    const double SF = M - Pv;
    const double PP = N + NM + Pv, MM = N - NM + Pv, PM = SF + CHI, MP = SF - CHI;
    obs[0] = N;
    obs[1] = M;
    obs[2] = NM;
    obs[3] = Pv;
    obs[4] = CHI;
    obs[5] = SF;
    obs[6] = PP;
    obs[7] = MM;
    obs[8] = PM;
    obs[9] = MP;
    obs[10] = PP + PM;
    obs[11] = MM + MP;
    obs[12] = 0.5 * (PP + MM + PM + MP);

    double *o = out + set * (int64_t)n_out * P + p;
    int row = 0;
    for (int b = 0; b < 13; ++b)
        if (mask & (1u << b)) {
            o[(int64_t)row * P] = obs[b];
            ++row;
        }
}

int launch_cross_section(const Detector &d, int64_t n_sets, const double *amp, const double *spec,
                         const numag_consts &c, uint32_t mask, double *out, hipStream_t s)
{
    const int64_t P = (int64_t)d.n0 * d.n1;
    const int64_t n = n_sets * P;
    if (n <= 0) return NUMAG_OK;
    const int n_out = __builtin_popcount(mask);
    hipLaunchKernelGGL(cross_section_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d,
                       n_sets, amp, spec, c, mask, n_out, out);
    NUMAG_HIP_CHECK(hipGetLastError());
    return NUMAG_OK;
}

// ---------------------------------------------------------------------------
// spectral (cross-correlation) matrices G_ab = A_a conj(A_b) of amplitude sets
// (Sec. 3.4 export of the Fourier cross-correlation functions, extended by the
// nuclear channel), packed as 16 reals per pixel.
// ---------------------------------------------------------------------------
// G = scale A A^H (accumulate: G += scale A A^H)
__global__ void spectral_matrix_kernel(int64_t n, const double *__restrict__ amp, double scale, int accumulate,
                                       double *__restrict__ G)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *A = amp + i * 8;
    double *g = G + i * 16;
    double v[16];
#pragma unroll
    for (int a = 0; a < 4; ++a) v[a] = A[2 * a] * A[2 * a] + A[2 * a + 1] * A[2 * a + 1];
    const int pa[6] = {0, 0, 0, 1, 1, 2};
    const int pb[6] = {1, 2, 3, 2, 3, 3};
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        const double ar = A[2 * pa[t]], ai = A[2 * pa[t] + 1];
        const double br = A[2 * pb[t]], bi = A[2 * pb[t] + 1];
        v[4 + 2 * t] = ar * br + ai * bi;  // Re(A_a conj(A_b))
        v[5 + 2 * t] = ai * br - ar * bi;  // Im(A_a conj(A_b))
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) g[e] = accumulate ? g[e] + scale * v[e] : scale * v[e];
}

int launch_spectral_matrix(int64_t n_sets, int64_t P, const double *amp, double *spec, hipStream_t s,
                           double scale, int accumulate)
{
    const int64_t n = n_sets * P;
    if (n <= 0) return NUMAG_OK;
    hipLaunchKernelGGL(spectral_matrix_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, amp, scale,
                       accumulate, spec);
    NUMAG_HIP_CHECK(hipGetLastError());
    return NUMAG_OK;
}

// ---------------------------------------------------------------------------
// azimuthal average
// ---------------------------------------------------------------------------
// Bin of a Cartesian pixel: floor(|q| / dq) with |q| = sqrt(qy*qy + qz*qz)
// (no fused operations), |q| == qmax_avg into the last bin, -1 if outside.
__device__ __forceinline__ int cart_bin(double qy, double qz, double dq, double qmax_avg, int n_bins)
{
#pragma clang fp contract(off)
    double a2 = qy * qy;
    double b2 = qz * qz;
    double qn = sqrt(a2 + b2);
    if (qn > qmax_avg) return -1;
    int b = (int)floor(qn / dq);
    if (b >= n_bins) b = n_bins - 1;
    return b;
}

constexpr int kAzThreads = 256;

// One workgroup per (data set, bin).  Candidate pixels are the bounding rows of
// the annulus and, per row, the two column intervals it can cover (widened by
// two columns); the exact bin test decides membership.
__global__ __launch_bounds__(kAzThreads) void azimuthal_cartesian_kernel(
    Detector d, const double *__restrict__ f, int n_bins, double qmax_avg, double *__restrict__ I,
    int64_t *__restrict__ count)
{
    const int b = blockIdx.x;
    const int set = blockIdx.y;
    const int64_t P = (int64_t)d.n0 * d.n1;
    const double *fs = f + (int64_t)set * P;
    const double dq = qmax_avg / (double)n_bins;
    const double r_in = (double)b * dq;
    const double r_out = (b == n_bins - 1) ? qmax_avg : (double)(b + 1) * dq;

    double sum = 0.0;
    long long cnt = 0;
    // index range of an axis covering [lo, hi] (with margin)
    auto idx_lo = [](double v, double origin, double step, int n) {
        if (step == 0.0) return 0;
        double x = floor((v - origin) / step) - 2.0;
        return (int)fmax(0.0, fmin((double)(n - 1), x));
    };
    auto idx_hi = [](double v, double origin, double step, int n) {
        if (step == 0.0) return n - 1;
        double x = ceil((v - origin) / step) + 2.0;
        return (int)fmax(0.0, fmin((double)(n - 1), x));
    };
    const int i_lo = idx_lo(-r_out, d.origin0, d.step0, d.n0);
    const int i_hi = idx_hi(r_out, d.origin0, d.step0, d.n0);
    for (int i = i_lo + (int)threadIdx.x; i <= i_hi; i += kAzThreads) {
        const double qy = axis_value(d.origin0, i, d.step0);
        const double y2 = qy * qy;
        const double c_out = sqrt(fmax(0.0, r_out * r_out - y2));
        const double c_in = (r_in * r_in > y2) ? sqrt(r_in * r_in - y2) : 0.0;
        // right interval [c_in, c_out] and left interval [-c_out, -c_in]
        for (int side = 0; side < 2; ++side) {
            const double lo = side == 0 ? c_in : -c_out;
            const double hi = side == 0 ? c_out : -c_in;
            int k_lo = idx_lo(lo, d.origin1, d.step1, d.n1);
            int k_hi = idx_hi(hi, d.origin1, d.step1, d.n1);
            if (side == 1) {
                // avoid visiting columns twice where the intervals overlap
                const int r_lo = idx_lo(c_in, d.origin1, d.step1, d.n1);
                if (k_hi >= r_lo) k_hi = r_lo - 1;
            }
            for (int k = k_lo; k <= k_hi; ++k) {
                const double qz = axis_value(d.origin1, k, d.step1);
                if (cart_bin(qy, qz, dq, qmax_avg, n_bins) == b) {
                    sum += fs[(int64_t)i * d.n1 + k];
                    ++cnt;
                }
            }
        }
    }
    __shared__ double s_sum[kAzThreads];
    __shared__ long long s_cnt[kAzThreads];
    s_sum[threadIdx.x] = sum;
    s_cnt[threadIdx.x] = cnt;
    __syncthreads();
    for (int w = kAzThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s_sum[threadIdx.x] += s_sum[threadIdx.x + w];
            s_cnt[threadIdx.x] += s_cnt[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const long long n = s_cnt[0];
        I[(int64_t)set * n_bins + b] = n > 0 ? s_sum[0] / (double)n : __builtin_nan("");
        if (count != nullptr && set == 0) count[b] = n;
    }
}

// One workgroup per (data set, q row): periodic trapezoid over theta.
__global__ __launch_bounds__(kAzThreads) void azimuthal_polar_kernel(Detector d,
                                                                     const double *__restrict__ f,
                                                                     int n_bins, double *__restrict__ I,
                                                                     int64_t *__restrict__ count)
{
    const int b = blockIdx.x;
    const int set = blockIdx.y;
    const int64_t P = (int64_t)d.n0 * d.n1;
    const double *row = f + (int64_t)set * P + (int64_t)b * d.n1;
    const double h = 2.0 * 3.141592653589793 / (double)d.n1;
    double sum = 0.0;
    for (int m = threadIdx.x; m < d.n1; m += kAzThreads) {
        const int m1 = (m + 1) % d.n1;
        sum += 0.5 * h * (row[m] + row[m1]);
    }
    __shared__ double s_sum[kAzThreads];
    s_sum[threadIdx.x] = sum;
    __syncthreads();
    for (int w = kAzThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s_sum[threadIdx.x] += s_sum[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        I[(int64_t)set * n_bins + b] = s_sum[0] / (2.0 * 3.141592653589793);
        if (count != nullptr && set == 0) count[b] = d.n1;
    }
}

int launch_azimuthal(const Detector &d, const double *f, int n_f, int n_bins, double qmax_avg,
                     double *I, int64_t *count, hipStream_t s)
{
    if (n_f <= 0 || n_bins <= 0) return NUMAG_OK;
    dim3 grid(n_bins, n_f);
    if (d.kind == NUMAG_GRID_CARTESIAN)
        hipLaunchKernelGGL(azimuthal_cartesian_kernel, grid, dim3(kAzThreads), 0, s, d, f, n_bins,
                           qmax_avg, I, count);
    else
        hipLaunchKernelGGL(azimuthal_polar_kernel, grid, dim3(kAzThreads), 0, s, d, f, n_bins, I, count);
    NUMAG_HIP_CHECK(hipGetLastError());
    return NUMAG_OK;
}

// ---------------------------------------------------------------------------
// correlation functions (trapezoid in the order of the samples)
// ---------------------------------------------------------------------------
__global__ void correlation_kernel(const double *__restrict__ q, const double *__restrict__ Iq, int n_q,
                                   int n_f, const double *__restrict__ r, int n_r, double scale,
                                   double *__restrict__ c, double *__restrict__ p)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_f * n_r) return;
    const int s = (int)(idx / n_r), t = (int)(idx % n_r);
    const double rt = r[t];
    double prev_q = 0.0, prev_y = 0.0, sum = 0.0;
    for (int b = 0; b < n_q; ++b) {
        const double Ib = Iq[(int64_t)s * n_q + b];
        if (isnan(Ib)) continue;
        const double x = q[b] * rt;
        const double j0 = (x == 0.0) ? 1.0 : sin(x) / x;
        const double y = Ib * q[b] * q[b] * j0;
        sum += 0.5 * (q[b] - prev_q) * (y + prev_y);
        prev_q = q[b];
        prev_y = y;
    }
    const double cv = scale * sum / (2.0 * 3.141592653589793 * 3.141592653589793);
    c[idx] = cv;
    p[idx] = rt * rt * cv;
}

int launch_correlation(const double *q, const double *I, int n_q, int n_f, const double *r, int n_r,
                       double scale, double *c, double *p, hipStream_t s)
{
    const int64_t n = (int64_t)n_f * n_r;
    if (n <= 0) return NUMAG_OK;
    hipLaunchKernelGGL(correlation_kernel, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, q, I, n_q,
                       n_f, r, n_r, scale, c, p);
    NUMAG_HIP_CHECK(hipGetLastError());
    return NUMAG_OK;
}

}  // namespace numag
