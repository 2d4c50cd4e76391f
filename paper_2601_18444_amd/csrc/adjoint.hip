// Gradient of a loss on the unpolarized cross section (Sec. 2.4) with respect
// to every input weight: the adjoint (transposed) Fourier sum on gfx950.
//
//   I_p = (scale/V)(|S_N|^2 + bH^2 |Q|^2),  Q = -Pp S_M,  L = sum_p w_p (I_p - T_p)^2
//   dL/dn_j   = Re sum_p a_N(p) exp(-i q_p . X_j),   a_N = 4 w r (scale/V) conj(S_N)
//   dL/dm'_ja = Re sum_p a_a(p) exp(-i q_p . X_j),   a_a = 4 w r (scale/V) bH^2 conj((Pp S_M)_a)
// with r = I_p - T_p and m' = R m (so dL/dm = R^T dL/dm').
//
// The adjoint sum swaps the roles of points and pixels: a lane owns a few
// points and walks the detector, row by row.  The row-start phasor is the
// previous row's times exp(-i dq_y Y) (one complex product), restarted from a
// fresh FP64 sincos every kAdjRowRestart rows (at most 2^7 ulp of drift); along
// the row the phasors follow the two-term recurrence
//     p_{c+1} = 2 cos(dq_z Z) p_c - p_{c-1}
// (two FMAs per column; an error made at column k reaches column c multiplied
// by at most c - k + 1, so a 256-column row keeps about 38 of the 53 bits in
// the worst case).  The residual weights of one row are staged in LDS and read
// as wave-wide broadcasts.  Ten FP64 VALU operations per (point, pixel) term.
#include "numag_internal.h"
#include "phasor.h"

namespace numag {

constexpr int kResThreads = 256;

// Residual weights a[p][4 complex] and per-block loss partials.
__global__ __launch_bounds__(kResThreads) void residual_kernel(Detector d, numag_consts k,
                                                               const double *__restrict__ amp,
                                                               const double *__restrict__ target,
                                                               const double *__restrict__ weight,
                                                               double *__restrict__ a,
                                                               double *__restrict__ loss_part)
{
    const int64_t P = (int64_t)d.n0 * d.n1;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double lp = 0.0;
    if (p < P) {
        double s, c;
        pixel_qhat(d, p, s, c);
        const double qh[3] = {0.0, s, c};
        const double *A = amp + p * 8;
        double Vr[3], Vi[3];
        for (int x = 0; x < 3; ++x) {
            double dot_r = qh[0] * A[2] + qh[1] * A[4] + qh[2] * A[6];
            double dot_i = qh[0] * A[3] + qh[1] * A[5] + qh[2] * A[7];
            Vr[x] = A[2 + 2 * x] - qh[x] * dot_r;
            Vi[x] = A[3 + 2 * x] - qh[x] * dot_i;
        }
        const double cf = k.scale / k.V;
        const double b2 = k.bH * k.bH;
        const double absV2 = Vr[0] * Vr[0] + Vi[0] * Vi[0] + Vr[1] * Vr[1] + Vi[1] * Vi[1] +
                             Vr[2] * Vr[2] + Vi[2] * Vi[2];
        const double I = cf * (A[0] * A[0] + A[1] * A[1] + b2 * absV2);
        // dL/dI_p: 2 w (I - T) for the built-in loss, or the caller's upstream
        // gradient (held in `weight`) when no target is given.
        double dLdI;
        if (target != nullptr) {
            const double r = I - target[p];
            const double w = weight[p];
            lp = w * r * r;
            dLdI = 2.0 * w * r;
        } else {
            dLdI = weight[p];
        }
        const double g = 2.0 * dLdI * cf;
        // polar: column-major [theta][q] so the adjoint stages a column contiguously
        const int64_t po = d.kind == NUMAG_GRID_CARTESIAN ? p : (p % d.n1) * d.n0 + p / d.n1;
        double *o = a + po * 8;
        o[0] = g * A[0];
        o[1] = -g * A[1];
        for (int x = 0; x < 3; ++x) {
            o[2 + 2 * x] = g * b2 * Vr[x];
            o[3 + 2 * x] = -g * b2 * Vi[x];
        }
    }
    __shared__ double s_l[kResThreads];
    s_l[threadIdx.x] = lp;
    __syncthreads();
    for (int w = kResThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s_l[threadIdx.x] += s_l[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = s_l[0];
}

__global__ void loss_sum_kernel(const double *__restrict__ part, int n, double *__restrict__ loss)
{
    __shared__ double s_l[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
    s_l[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s_l[threadIdx.x] += s_l[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = s_l[0];
}

constexpr int kAdjThreads = 256;
constexpr int kAdjNPL = 4;      // points per lane
constexpr int kAdjMaxCols = 256;  // columns staged per LDS pass
constexpr int kAdjRowRestart = 64;  // rows between fresh row-start phasors

// grid.x: point blocks of kAdjThreads * kAdjNPL; grid.y: row ranges.
// Residual weights of one column as the adjoint reads them (from LDS).
struct ColW {
    double a0r, a0i, a1r, a1i, a2r, a2i, a3r, a3i;
};

__device__ __forceinline__ ColW load_col(const double *p)
{
    return ColW{p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7]};
}

// One column for the lane's points: Re(a p) (two FMAs per channel), then the
// recurrence step to the next column.
__device__ __forceinline__ void adjoint_column(const ColW &w, double2 (&pc)[kAdjNPL], double2 (&pm)[kAdjNPL],
                                               const double (&kz)[kAdjNPL], double (&acc)[kAdjNPL][4])
{
#pragma unroll
    for (int u = 0; u < kAdjNPL; ++u) {
        const double2 p = pc[u];
        acc[u][0] = fma(-w.a0i, p.y, fma(w.a0r, p.x, acc[u][0]));
        acc[u][1] = fma(-w.a1i, p.y, fma(w.a1r, p.x, acc[u][1]));
        acc[u][2] = fma(-w.a2i, p.y, fma(w.a2r, p.x, acc[u][2]));
        acc[u][3] = fma(-w.a3i, p.y, fma(w.a3r, p.x, acc[u][3]));
        pc[u] = make_double2(fma(kz[u], p.x, -pm[u].x), fma(kz[u], p.y, -pm[u].y));
        pm[u] = p;
    }
}

// The detector rows of the split are walked as segments of at most kAdjMaxCols
// columns.  While a segment is summed from one LDS buffer, each thread holds the
// next segment's residual weights in registers (loaded at the segment's start)
// and stores them into the other buffer afterwards: one barrier per segment and
// the global-memory latency hidden behind the sums.  Within a segment the
// weights of column k + 1 are read from LDS before column k is summed.
constexpr int kAdjPer = kAdjMaxCols * 8 / kAdjThreads;  // doubles per thread per segment
static_assert(kAdjPer * kAdjThreads == kAdjMaxCols * 8, "segment split over the threads");

__global__ __launch_bounds__(kAdjThreads, 2) void adjoint_cartesian_kernel(
    const PointRec *__restrict__ pts, int64_t W, Detector d, const double *__restrict__ a,
    int rows_per_split, double *__restrict__ gpart)
{
    __shared__ double s_a[2][kAdjMaxCols * 8];
    const int64_t jb = (int64_t)blockIdx.x * kAdjThreads * kAdjNPL + threadIdx.x;
    const int r0 = blockIdx.y * rows_per_split;
    const int r1 = min(d.n0, r0 + rows_per_split);
    const int segs = (d.n1 + kAdjMaxCols - 1) / kAdjMaxCols;  // segments per row
    const int nseg = (r1 - r0) * segs;

    double Y[kAdjNPL], Z[kAdjNPL], kz[kAdjNPL];
    double2 ez0[kAdjNPL], dzc[kAdjNPL], ey[kAdjNPL], dy[kAdjNPL];
    double acc[kAdjNPL][4];
    const double qz0 = axis_value(d.origin1, 0, d.step1);
#pragma unroll
    for (int u = 0; u < kAdjNPL; ++u) {
        const int64_t j = jb + (int64_t)u * kAdjThreads;
        const bool ok = j < W;
        Y[u] = ok ? pts[j].Y : 0.0;
        Z[u] = ok ? pts[j].Z : 0.0;
        ez0[u] = twiddle(qz0 * Z[u]);
        const double2 dz = twiddle(d.step1 * Z[u]);
        dzc[u] = make_double2(dz.x, -dz.y);  // inverse column step
        kz[u] = dz.x + dz.x;
        dy[u] = twiddle(d.step0 * Y[u]);     // row step
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    }

    // residual weights of segment g (row r0 + g / segs, columns from (g % segs) kAdjMaxCols)
    auto fetch = [&](int g, double (&reg)[kAdjPer]) {
        const int row = r0 + g / segs, c0 = (g % segs) * kAdjMaxCols;
        const int nc = min(kAdjMaxCols, d.n1 - c0);
        const double *src = a + ((int64_t)row * d.n1 + c0) * 8;
#pragma unroll
        for (int e = 0; e < kAdjPer; ++e) {
            const int i = threadIdx.x + e * kAdjThreads;
            reg[e] = i < nc * 8 ? src[i] : 0.0;
        }
    };
    double reg[kAdjPer];
    if (nseg > 0) {
        fetch(0, reg);
#pragma unroll
        for (int e = 0; e < kAdjPer; ++e) s_a[0][threadIdx.x + e * kAdjThreads] = reg[e];
    }
    __syncthreads();

    double2 pc[kAdjNPL], pm[kAdjNPL];  // phasors of the current column and of the one before
    for (int g = 0; g < nseg; ++g) {
        const int buf = g & 1;
        if (g + 1 < nseg) fetch(g + 1, reg);
        const int c0 = (g % segs) * kAdjMaxCols;
        const int nc = min(kAdjMaxCols, d.n1 - c0);
        if (c0 == 0) {  // row start: fresh column phasors
            const int rr = g / segs;  // row within the split
            if (rr % kAdjRowRestart == 0) {
                const double qy = axis_value(d.origin0, r0 + rr, d.step0);
#pragma unroll
                for (int u = 0; u < kAdjNPL; ++u) ey[u] = twiddle(qy * Y[u]);
            }
#pragma unroll
            for (int u = 0; u < kAdjNPL; ++u) {
                pc[u] = cmul(ey[u], ez0[u]);
                pm[u] = cmul(pc[u], dzc[u]);
                ey[u] = cmul(ey[u], dy[u]);  // next row
            }
        }
        const double *sa = s_a[buf];
        ColW wa = load_col(sa);
        int k = 0;
        for (; k + 1 < nc; k += 2) {
            const ColW wb = load_col(sa + (k + 1) * 8);
            __builtin_amdgcn_sched_barrier(0);
            adjoint_column(wa, pc, pm, kz, acc);
            __builtin_amdgcn_sched_barrier(0);
            wa = load_col(sa + min(k + 2, nc - 1) * 8);
            __builtin_amdgcn_sched_barrier(0);
            adjoint_column(wb, pc, pm, kz, acc);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (k < nc) adjoint_column(wa, pc, pm, kz, acc);
        if (g + 1 < nseg) {
#pragma unroll
            for (int e = 0; e < kAdjPer; ++e) s_a[buf ^ 1][threadIdx.x + e * kAdjThreads] = reg[e];
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < kAdjNPL; ++u) {
        const int64_t j = jb + (int64_t)u * kAdjThreads;
        if (j < W) {
            double *o = gpart + ((int64_t)blockIdx.y * W + j) * 4;
#pragma unroll
            for (int v = 0; v < 4; ++v) o[v] = acc[u][v];
        }
    }
}

// Polar detector: phase q_i u_m with u_m = Y sin(theta_m) + Z cos(theta_m).  A lane
// owns kAdjNPL points; per theta column it forms u, the q step exp(-i dq u) (one
// sincos) and walks the q rows with the two-term recurrence, restarted from a
// fresh sincos every kPolRestart rows (the error growth of the recurrence stays
// below kPolRestart^2 / 2 ulp, 2^15 ulp or 7e-12 relative; the first segment starts
// at q = 0, whose phasor is 1 without a sincos).  The residual weights are column-major
// [theta][q][8] and are walked as segments of kPolRestart rows of one column,
// double-buffered in LDS like the Cartesian kernel's: the next segment is held
// in registers while the current one is summed.
// grid.x: point blocks of kAdjThreads * kAdjNPL; grid.y: theta-column ranges.
constexpr int kPolRestart = 256;
constexpr int kPolPer = kPolRestart * 8 / kAdjThreads;  // doubles per thread per segment
static_assert(kPolPer * kAdjThreads == kPolRestart * 8, "segment split over the threads");

__global__ __launch_bounds__(kAdjThreads, 2) void adjoint_polar_kernel(
    const PointRec *__restrict__ pts, int64_t W, Detector d, const double *__restrict__ a, int cols_per_split,
    double *__restrict__ gpart)
{
    __shared__ double s_a[2][kPolRestart * 8];
    const int64_t jb = (int64_t)blockIdx.x * kAdjThreads * kAdjNPL + threadIdx.x;
    const int c0 = blockIdx.y * cols_per_split;
    const int c1 = min(d.n1, c0 + cols_per_split);
    const int rsegs = (d.n0 + kPolRestart - 1) / kPolRestart;  // segments per column
    const int nseg = max(0, c1 - c0) * rsegs;

    double Y[kAdjNPL], Z[kAdjNPL];
    double acc[kAdjNPL][4];
#pragma unroll
    for (int u = 0; u < kAdjNPL; ++u) {
        const int64_t j = jb + (int64_t)u * kAdjThreads;
        const bool ok = j < W;
        Y[u] = ok ? pts[j].Y : 0.0;
        Z[u] = ok ? pts[j].Z : 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    }

    // residual weights of segment g (column c0 + g / rsegs, rows from (g % rsegs) kPolRestart)
    auto fetch = [&](int g, double (&reg)[kPolPer]) {
        const int col = c0 + g / rsegs, r0 = (g % rsegs) * kPolRestart;
        const int nr = min(kPolRestart, d.n0 - r0);
        const double *src = a + ((int64_t)col * d.n0 + r0) * 8;
#pragma unroll
        for (int e = 0; e < kPolPer; ++e) {
            const int i = threadIdx.x + e * kAdjThreads;
            reg[e] = i < nr * 8 ? src[i] : 0.0;
        }
    };
    double reg[kPolPer];
    if (nseg > 0) {
        fetch(0, reg);
#pragma unroll
        for (int e = 0; e < kPolPer; ++e) s_a[0][threadIdx.x + e * kAdjThreads] = reg[e];
    }
    __syncthreads();

    double uu[kAdjNPL], kq[kAdjNPL];
    double2 stc[kAdjNPL];  // inverse q step exp(+i dq u)
    for (int g = 0; g < nseg; ++g) {
        const int buf = g & 1;
        if (g + 1 < nseg) fetch(g + 1, reg);
        const int col = c0 + g / rsegs, r0 = (g % rsegs) * kPolRestart;
        const int nr = min(kPolRestart, d.n0 - r0);
        if (r0 == 0) {  // new column: u and the q step of every point
            const double th = (2.0 * 3.141592653589793 * (double)col) / (double)d.n_theta;
            double sth, cth;
            sincos(th, &sth, &cth);
#pragma unroll
            for (int u = 0; u < kAdjNPL; ++u) {
                uu[u] = Y[u] * sth + Z[u] * cth;
                const double2 st = twiddle(d.step0 * uu[u]);
                stc[u] = make_double2(st.x, -st.y);
                kq[u] = st.x + st.x;
            }
        }
        // recurrence restart at row r0: phasors of rows r0 and r0 - 1
        const double q0 = axis_value(0.0, r0, d.step0);
        double2 pc[kAdjNPL], pm[kAdjNPL];
#pragma unroll
        for (int u = 0; u < kAdjNPL; ++u) {
            pc[u] = r0 == 0 ? make_double2(1.0, 0.0) : twiddle(q0 * uu[u]);
            pm[u] = cmul(pc[u], stc[u]);
        }
        const double *sa = s_a[buf];
#pragma unroll 2
        for (int i = 0; i < nr; ++i) {
            const double *ai = sa + i * 8;
            const double a0r = ai[0], a0i = ai[1], a1r = ai[2], a1i = ai[3];
            const double a2r = ai[4], a2i = ai[5], a3r = ai[6], a3i = ai[7];
#pragma unroll
            for (int u = 0; u < kAdjNPL; ++u) {
                const double2 p = pc[u];
                acc[u][0] = fma(-a0i, p.y, fma(a0r, p.x, acc[u][0]));
                acc[u][1] = fma(-a1i, p.y, fma(a1r, p.x, acc[u][1]));
                acc[u][2] = fma(-a2i, p.y, fma(a2r, p.x, acc[u][2]));
                acc[u][3] = fma(-a3i, p.y, fma(a3r, p.x, acc[u][3]));
                pc[u] = make_double2(fma(kq[u], p.x, -pm[u].x), fma(kq[u], p.y, -pm[u].y));
                pm[u] = p;
            }
        }
        if (g + 1 < nseg) {
#pragma unroll
            for (int e = 0; e < kPolPer; ++e) s_a[buf ^ 1][threadIdx.x + e * kAdjThreads] = reg[e];
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < kAdjNPL; ++u) {
        const int64_t j = jb + (int64_t)u * kAdjThreads;
        if (j < W) {
            double *o = gpart + ((int64_t)blockIdx.y * W + j) * 4;
#pragma unroll
            for (int v = 0; v < 4; ++v) o[v] = acc[u][v];
        }
    }
}

__global__ void grad_finalize_kernel(const double *__restrict__ gpart, int nsplit, int64_t W, Rot R,
                                     double *__restrict__ dnuc, double *__restrict__ dmag)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= W) return;
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < nsplit; ++s)
        for (int v = 0; v < 4; ++v) g[v] += gpart[((int64_t)s * W + j) * 4 + v];
    if (dnuc != nullptr) dnuc[j] = g[0];
    if (dmag != nullptr) {
        for (int b = 0; b < 3; ++b)
            dmag[3 * j + b] = R.m[0 * 3 + b] * g[1] + R.m[1 * 3 + b] * g[2] + R.m[2 * 3 + b] * g[3];
    }
}

// Ranges the detector is split into (rows on a Cartesian detector, theta
// columns on a polar one), so that point blocks x ranges fill the chip.
static int adjoint_row_splits(const Detector &d, int64_t W)
{
    int64_t pblocks = (W + kAdjThreads * kAdjNPL - 1) / (kAdjThreads * kAdjNPL);
    if (pblocks < 1) pblocks = 1;
    const int64_t target = current_tune_shape(kTuneAdjoint, d, W).target;
    int64_t want = (target + pblocks - 1) / pblocks;
    const int extent = d.kind == NUMAG_GRID_CARTESIAN ? d.n0 : d.n1;
    if (want > extent) want = extent;
    if (want < 1) want = 1;
    return (int)want;
}

// The part of the detector the adjoint sums: the whole detector, or the half of the
// Hermitian path (Cartesian rows [0, ceil(n0 / 2)), polar columns [0, n_theta / 2);
// d.n_theta stays that of the whole detector).
static Detector adjoint_detector(const Detector &d_full, bool hermitian)
{
    Detector d = d_full;
    if (hermitian) {
        if (d.kind == NUMAG_GRID_CARTESIAN)
            d.n0 = (d.n0 + 1) / 2;
        else
            d.n1 = d.n1 / 2;
    }
    return d;
}

// Scratch of launch_grad: the residual weights and loss partials of the whole
// detector, and the gradient partials of the row splits of the part the adjoint
// sums (its launch shape, hence its split count, is looked up for that part).
size_t grad_workspace_bytes(const Detector &d_full, int64_t W, bool hermitian)
{
    const int64_t P = (int64_t)d_full.n0 * d_full.n1;
    const int64_t nres = (P + kResThreads - 1) / kResThreads;
    const int splits = adjoint_row_splits(adjoint_detector(d_full, hermitian), W);
    size_t b = 0;
    b += (size_t)P * 8 * sizeof(double);          // residual weights
    b += (size_t)(nres + 1) * sizeof(double);      // loss partials
    b += (size_t)splits * (size_t)W * 4 * sizeof(double);
    return b + 3 * 256;
}

// Residual weights folded onto half of a detector that is symmetric about q = 0:
// the term of the mirror pixel p' (at -q_p within an ulp) is
// Re[a(p') exp(+i q_p X)] = Re[conj a(p') exp(-i q_p X)], so the adjoint over the
// half with a(p) + conj a(p') equals the full one, whatever the target and the
// loss weights.  Cartesian: p' = P - 1 - p for p < Ph (pixels whose mirror lies
// in the half, the middle row of an odd n0, keep their own weight); polar
// (column-major [theta][q], even n_theta): p' = p + Ph.
__global__ void fold_residual_kernel(double *__restrict__ a, int64_t P, int64_t Ph, int polar)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Ph * 8) return;
    const int64_t p = idx >> 3;
    const int v = (int)(idx & 7);
    const int64_t q = polar ? p + Ph : P - 1 - p;
    if (q < Ph) return;
    a[idx] += (v & 1) ? -a[q * 8 + v] : a[q * 8 + v];
}

int launch_grad(const PointRec *pts, int64_t W, const Detector &d_full, const numag_consts &c,
                const double *amp, const double *target, const double *weight, double *loss,
                double *dnuc, double *dmag, const Rot &R, void *ws, size_t ws_bytes, hipStream_t s,
                bool hermitian)
{
    const Detector &dr = d_full;  // the residual and the loss cover the whole detector
    const int64_t P = (int64_t)dr.n0 * dr.n1;
    const int64_t nres = (P + kResThreads - 1) / kResThreads;
    // the adjoint sums the whole detector, or half of it with folded weights; the
    // split count is the one grad_workspace_bytes sized the scratch for
    const Detector d = adjoint_detector(d_full, hermitian);
    const int splits = adjoint_row_splits(d, W);
    char *base = (char *)ws;
    auto take = [&](size_t bytes) {
        char *r = base;
        base += (bytes + 255) & ~(size_t)255;
        return r;
    };
    double *a = (double *)take((size_t)P * 8 * sizeof(double));
    double *lpart = (double *)take((size_t)(nres + 1) * sizeof(double));
    double *gpart = (double *)take((size_t)splits * (size_t)W * 4 * sizeof(double));
    if ((size_t)(base - (char *)ws) > ws_bytes) {
        set_error("numag_grad: workspace too small");
        return NUMAG_E_WORKSPACE;
    }
    hipLaunchKernelGGL(residual_kernel, dim3((unsigned)nres), dim3(kResThreads), 0, s, dr, c, amp, target,
                       weight, a, lpart);
    NUMAG_HIP_CHECK(hipGetLastError());
    if (loss != nullptr) {
        hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(256), 0, s, lpart, (int)nres, loss);
        NUMAG_HIP_CHECK(hipGetLastError());
    }
    if (W <= 0) return NUMAG_OK;
    if (hermitian) {
        const int64_t Ph = (int64_t)d.n0 * d.n1;
        hipLaunchKernelGGL(fold_residual_kernel, dim3((unsigned)((Ph * 8 + 255) / 256)), dim3(256), 0, s, a, P, Ph,
                           d.kind == NUMAG_GRID_POLAR ? 1 : 0);
        NUMAG_HIP_CHECK(hipGetLastError());
    }
    const int extent = d.kind == NUMAG_GRID_CARTESIAN ? d.n0 : d.n1;
    const int per = (extent + splits - 1) / splits;
    const int nsplit = (extent + per - 1) / per;
    const int64_t pblocks = (W + kAdjThreads * kAdjNPL - 1) / (kAdjThreads * kAdjNPL);
    {
        TimedLaunch timed(NUMAG_KERNEL_ADJOINT, s);
        if (d.kind == NUMAG_GRID_CARTESIAN)
            hipLaunchKernelGGL(adjoint_cartesian_kernel, dim3((unsigned)pblocks, nsplit), dim3(kAdjThreads), 0, s,
                               pts, W, d, a, per, gpart);
        else
            hipLaunchKernelGGL(adjoint_polar_kernel, dim3((unsigned)pblocks, nsplit), dim3(kAdjThreads), 0, s, pts,
                               W, d, a, per, gpart);
    }
    NUMAG_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(grad_finalize_kernel, dim3((unsigned)((W + 255) / 256)), dim3(256), 0, s, gpart,
                       nsplit, W, R, dnuc, dmag);
    NUMAG_HIP_CHECK(hipGetLastError());
    return NUMAG_OK;
}

}  // namespace numag
