// Two-dimensional correlation function (Sec. 2.6 eq. crav2d) and the angular
// spectrum (Sec. 2.5 eqs. CosineSinceIntensities, ModalAmplitudes) on gfx950.
//
// C(r) = int int f(q, theta) exp(i q rho cos(theta - alpha)) q dq dtheta is, with
// q = q (sin theta, cos theta) and r = rho (sin alpha, cos alpha) in the detector
// plane, the quadrature sum over detector pixels p
//     C(r) = sum_p wq_p f_p exp(i q_p . r),
// wq the trapezoidal weights (h_i q_i dtheta on the polar detector, dq_y dq_z
// with halved edges on a Cartesian one).  That is a direct Fourier sum whose
// "points" are the pixels, placed at -q_p so that the sums' exp(-i ...) becomes
// exp(+i q.r), with real weights wq_p f_p; the real-space grid plays the role of
// the detector.  It therefore runs on the same Cartesian / polar direct-sum
// kernels, and their weight channels carry up to four data sets at once: one set
// runs alone in channel 0 (the kernels' one-channel form, 4.5 instead of 10.5
// instructions per term), two or three in channels 1-3, four in all four.
#include <algorithm>

#include "numag_internal.h"
#include "phasor.h"

namespace numag {


// Pixels of detector d as points: Y = -q_y, Z = -q_z, weight channel c0 + c =
// wq * f_(set0 + c), the other channels zero.
__global__ void corr2d_points_kernel(Detector d, const double *__restrict__ f, int n_f, int set0, int c0,
                                     PointRec *__restrict__ out)
{
    const int64_t P = (int64_t)d.n0 * d.n1;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int row = (int)(p / d.n1), col = (int)(p % d.n1);
    double qy, qz, wq;
    if (d.kind == NUMAG_GRID_CARTESIAN) {
        qy = axis_value(d.origin0, row, d.step0);
        qz = axis_value(d.origin1, col, d.step1);
        const double cy = (row == 0 || row == d.n0 - 1) ? 0.5 : 1.0;
        const double cz = (col == 0 || col == d.n1 - 1) ? 0.5 : 1.0;
        const double dy = d.n0 > 1 ? d.step0 : 1.0, dz = d.n1 > 1 ? d.step1 : 1.0;
        wq = cy * cz * dy * dz;
    } else {
        const double q = axis_value(0.0, row, d.step0);
        const double th = (2.0 * 3.141592653589793 * (double)col) / (double)d.n1;
        double s, c;
        sincos(th, &s, &c);
        qy = q * s;
        qz = q * c;
        const double h = (row == 0 || row == d.n0 - 1) ? 0.5 * d.step0 : d.step0;
        wq = h * q * (2.0 * 3.141592653589793 / (double)d.n1);
    }
    PointRec r;
    r.Y = -qy;
    r.Z = -qz;
    for (int c = 0; c < 4; ++c) {
        const int set = set0 + c - c0;
        r.w[c] = (c >= c0 && set < n_f) ? wq * f[(int64_t)set * P + p] : 0.0;
    }
    r.pad[0] = r.pad[1] = 0.0;
    out[p] = r;
}

// C_out[set0 + c][t] = channel c0 + c of amp[t]
__global__ void corr2d_scatter_kernel(const double *__restrict__ amp, int64_t R, int n_f, int set0, int c0,
                                      double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= R * 4) return;
    const int64_t t = i / 4;
    const int c = (int)(i % 4);
    if (set0 + c >= n_f || c0 + c >= 4) return;
    double *o = out + ((int64_t)(set0 + c) * R + t) * 2;
    o[0] = amp[t * 8 + 2 * (c0 + c)];
    o[1] = amp[t * 8 + 2 * (c0 + c) + 1];
}

static size_t al2(size_t b) { return (b + 255) & ~(size_t)255; }

// The real-space grid to evaluate: C(-r) = conj C(r) for real data, so only half
// of a grid symmetric about r = 0 is summed (Cartesian: rows [0, ceil(n0/2));
// polar with an even n_alpha: columns [0, n_alpha/2)) and the rest is mirrored.
static Detector half_grid(const Detector &rd)
{
    Detector rh = rd;
    if (rd.kind == NUMAG_GRID_CARTESIAN)
        rh.n0 = (rd.n0 + 1) / 2;
    else if (rd.n1 % 2 == 0)
        rh.n1 = rd.n1 / 2;
    return rh;
}

static DirectPlan corr2d_plan(const Detector &rh, int64_t P)
{
    return rh.kind == NUMAG_GRID_CARTESIAN ? plan_direct_cartesian(rh, P) : plan_direct_polar(rh, P);
}

size_t correlation_2d_workspace_bytes(const Detector &d, const Detector &rd)
{
    const int64_t P = (int64_t)d.n0 * d.n1;
    const int64_t R = (int64_t)rd.n0 * rd.n1;
    const Detector rh = half_grid(rd);
    return al2((size_t)P * sizeof(PointRec)) + al2(direct_partial_bytes(corr2d_plan(rh, P), rh)) +
           al2((size_t)R * 8 * sizeof(double));
}
int launch_correlation_2d(const Detector &d, const double *f, int n_f, const Detector &rd, double *C, void *ws,
                          size_t ws_bytes, hipStream_t s)
{
    const int64_t P = (int64_t)d.n0 * d.n1;
    const int64_t R = (int64_t)rd.n0 * rd.n1;
    if (ws_bytes < correlation_2d_workspace_bytes(d, rd)) {
        set_error("numag_correlation_2d: workspace too small");
        return NUMAG_E_WORKSPACE;
    }
    const Detector rh = half_grid(rd);
    const int64_t Rh = (int64_t)rh.n0 * rh.n1;
    const DirectPlan plan4 = corr2d_plan(rh, P);
    char *base = (char *)ws;
    PointRec *pts = (PointRec *)base;
    double *part = (double *)(base + al2((size_t)P * sizeof(PointRec)));
    double *amp = (double *)(base + al2((size_t)P * sizeof(PointRec)) + al2(direct_partial_bytes(plan4, rh)));
    for (int set0 = 0; set0 < n_f; set0 += 4) {
        // the sum kernels' channel set for this group: 1 (channel 0), 3 (channels 1-3) or 4
        const int m = std::min(4, n_f - set0);
        DirectPlan plan = plan4;
        plan.channels = m == 1 ? 1 : (m == 4 ? 4 : 3);
        const int c0 = plan.channels == 3 ? 1 : 0;
        hipLaunchKernelGGL(corr2d_points_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, d, f, n_f, set0,
                           c0, pts);
        NUMAG_HIP_CHECK(hipGetLastError());
        int rc;
        if (rd.kind == NUMAG_GRID_CARTESIAN) {
            rc = launch_direct_cartesian(pts, P, rh, plan, plan.nsplit > 1 ? part : amp, s);
            if (rc == NUMAG_OK && plan.nsplit > 1) rc = launch_combine(part, plan.nsplit, Rh, amp, 0, s);
            if (rc == NUMAG_OK) rc = launch_mirror_cartesian(amp, R, Rh, s);
        } else {
            rc = launch_direct_polar(pts, P, rh, plan, part, s);
            if (rc == NUMAG_OK)
                rc = rh.n1 != rd.n1 ? launch_combine_polar_half(part, plan.nsplit, rd.n0, rh.n1, amp, s)
                                    : launch_combine(part, plan.nsplit, R, amp, 0, s);
        }
        if (rc != NUMAG_OK) return rc;
        hipLaunchKernelGGL(corr2d_scatter_kernel, dim3((unsigned)((R * 4 + 255) / 256)), dim3(256), 0, s, amp, R, n_f,
                           set0, c0, C);
        NUMAG_HIP_CHECK(hipGetLastError());
    }
    return NUMAG_OK;
}

// ---------------------------------------------------------------------------
// Angular spectrum on the polar detector: periodic trapezoid over theta of
// f sin(k theta), f cos(k theta) with prefactor (2 - delta_k0) / (2 pi).
// One workgroup per (data set, q row); thread k handles one order.
// ---------------------------------------------------------------------------
__global__ void angular_spectrum_kernel(Detector d, const double *__restrict__ f, int k_max,
                                        double *__restrict__ Is, double *__restrict__ Ic)
{
    const int row = blockIdx.x, set = blockIdx.y;
    const int64_t P = (int64_t)d.n0 * d.n1;
    const double *fr = f + (int64_t)set * P + (int64_t)row * d.n1;
    const double h = 2.0 * 3.141592653589793 / (double)d.n1;
    for (int k = threadIdx.x; k <= k_max; k += blockDim.x) {
        double ss = 0.0, cc = 0.0;
        for (int m = 0; m < d.n1; ++m) {
            const int m1 = (m + 1) % d.n1;
            double s0, c0, s1, c1;
            sincos((double)k * (h * (double)m), &s0, &c0);
            sincos((double)k * (h * (double)(m + 1)), &s1, &c1);
            ss += 0.5 * h * (fr[m] * s0 + fr[m1] * s1);
            cc += 0.5 * h * (fr[m] * c0 + fr[m1] * c1);
        }
        const double pref = (k == 0 ? 1.0 : 2.0) / (2.0 * 3.141592653589793);
        const int64_t o = ((int64_t)set * d.n0 + row) * (k_max + 1) + k;
        Is[o] = pref * ss;
        Ic[o] = pref * cc;
    }
}

// a_k = sum_i I_k(q_i);  A_k = a_k / sum_j sqrt(a_s_j^2 + a_c_j^2).  One thread per data set.
__global__ void modal_amplitude_kernel(const double *__restrict__ Is, const double *__restrict__ Ic, int n_q,
                                       int k_max, int n_f, double *__restrict__ As, double *__restrict__ Ac)
{
    const int set = blockIdx.x * blockDim.x + threadIdx.x;
    if (set >= n_f) return;
    double norm = 0.0;
    for (int k = 0; k <= k_max; ++k) {
        double as = 0.0, ac = 0.0;
        for (int i = 0; i < n_q; ++i) {
            as += Is[((int64_t)set * n_q + i) * (k_max + 1) + k];
            ac += Ic[((int64_t)set * n_q + i) * (k_max + 1) + k];
        }
        As[(int64_t)set * (k_max + 1) + k] = as;
        Ac[(int64_t)set * (k_max + 1) + k] = ac;
        norm += sqrt(as * as + ac * ac);
    }
    for (int k = 0; k <= k_max; ++k) {
        As[(int64_t)set * (k_max + 1) + k] /= norm;
        Ac[(int64_t)set * (k_max + 1) + k] /= norm;
    }
}

int launch_angular_spectrum(const Detector &d, const double *f, int n_f, int k_max, double *Is, double *Ic,
                            double *As, double *Ac, hipStream_t s)
{
    if (n_f <= 0) return NUMAG_OK;
    hipLaunchKernelGGL(angular_spectrum_kernel, dim3(d.n0, n_f), dim3(64), 0, s, d, f, k_max, Is, Ic);
    NUMAG_HIP_CHECK(hipGetLastError());
    if (As != nullptr && Ac != nullptr) {
        hipLaunchKernelGGL(modal_amplitude_kernel, dim3((n_f + 63) / 64), dim3(64), 0, s, Is, Ic, d.n0, k_max, n_f,
                           As, Ac);
        NUMAG_HIP_CHECK(hipGetLastError());
    }
    return NUMAG_OK;
}

}  // namespace numag
