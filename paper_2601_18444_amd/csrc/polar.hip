// Direct Fourier sums on the paper's polar (q, theta) detector (Sec. 3.2):
// S_c(q_i, theta_m) = sum_j w_{j,c} exp(-i q_i u_m(j)),  u_m = Y sin(theta_m) + Z cos(theta_m).
#include "cartesian_sum.h"

namespace numag {


// ---------------------------------------------------------------------------
// Polar direct sum.  The phase q_i u_m with u_m = Y sin(theta_m) + Z cos(theta_m)
// does not separate, but along q it is a geometric sequence: lanes own theta
// columns and each walks 8 q rows, the first by the row-group start, the second
// by one step exp(-i dq u), the rest by the two-term recurrence
// p_{r+1} = 2 cos(dq u) p_r - p_{r-1}.  A workgroup of WV waves covers 8 WV rows,
// so the per-(point, column) generation (u, one sincos for the step, the block
// start exp(-i q(row0) u) as a power of the step, the wave starts by the same
// recurrence with step^8) is shared by 8 WV rows.
// ---------------------------------------------------------------------------
constexpr int kPolarChunk = 8;
constexpr int kPolarB = 8;

// Operands of point jj for this lane: ez = the wave's start phasor, dz = the q step
// (the recurrence coefficient 2 Re dz is formed where it is used).
template <int WV, int R>
__device__ __forceinline__ cart::Operands polar_operands(const double2 (&s_start)[R][WV][64],
                                                         const double2 (&s_step)[R][64],
                                                         const double (&s_w)[R][4], int jj, int lane,
                                                         int wave)
{
    cart::Operands o;
    o.ez = s_start[jj][wave][lane];
    o.dz = s_step[jj][lane];
    o.k = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) o.w[v] = s_w[jj][v];
    return o;
}

// Adds one point to the lane's B q rows: start, one step, then the recurrence.
template <int B, int CH>
__device__ __forceinline__ void polar_point(const cart::Operands &o, double (&acc)[B][2 * CH])
{
    const double k = o.dz.x + o.dz.x;
    double2 pm = o.ez;
    double2 pc = cmul(pm, o.dz);
    cart::add_weighted<CH>(o, pm, acc[0]);
    cart::add_weighted<CH>(o, pc, acc[1]);
#pragma unroll
    for (int r = 2; r < B; ++r) {
        const double2 pn = make_double2(fma(k, pc.x, -pm.x), fma(k, pc.y, -pm.y));
        cart::add_weighted<CH>(o, pn, acc[r]);
        pm = pc;
        pc = pn;
    }
}

// LDS buffers of the polar kernel: two at WV = 8 (the next chunk is generated into
// one while the other is summed, one barrier per chunk, 149 KB), one at WV = 4
// (two workgroups per CU).
template <int WV>
constexpr int polar_buffers()
{
    return WV == 8 ? 2 : 1;
}

// grid.z = rotation r of a group x split sp (nsp splits per rotation); the points of
// rotation r are pts[r wrot, (r + 1) wrot).  One rotation: wrot = W, nsp = grid.z.
template <int WV, int CH>
__global__ __launch_bounds__(64 * WV, 8 / WV) void direct_polar_kernel(const PointRec *__restrict__ pts,
                                                                      int64_t wrot, int64_t per, int nsp, Detector d,
                                                                      double *__restrict__ out)
{
    constexpr int B = kPolarB;
    constexpr int ROWS = WV * B;
    constexpr int CHK = kPolarChunk;
    constexpr int NB = polar_buffers<WV>();
    // one row per point of a chunk; single-buffered, plus one the pipelined loop
    // may read past the end (double-buffered, that read is clamped instead)
    constexpr int R = NB == 2 ? CHK : CHK + 1;
    __shared__ double2 s_start[NB][R][WV][64];
    __shared__ double2 s_step[NB][R][64];
    __shared__ double s_w[NB][R][4];
    __shared__ double2 s_trig[64];  // (sin, cos) of the lane's column angle

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int col0 = blockIdx.x * 64;
    const int row0 = blockIdx.y * ROWS;
    const int64_t rbase = (int64_t)(blockIdx.z / nsp) * wrot;
    const int64_t jbeg = rbase + (int64_t)(blockIdx.z % nsp) * per;
    const int64_t jend = min(rbase + wrot, jbeg + per);

    double acc[B][2 * CH];
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
        for (int v = 0; v < 2 * CH; ++v) acc[r][v] = 0.0;

    // generation role: thread t handles column (t & 63) for points wave, wave + WV, ...
    const int gcol = col0 + lane;
    if (wave == 0) {
        const double theta = (2.0 * 3.141592653589793 * (double)gcol) / (double)d.n_theta;
        double sth, cth;
        sincos(theta, &sth, &cth);
        s_trig[lane] = make_double2(sth, cth);
    }
    __syncthreads();
    const double qrow0 = axis_value(d.origin0, row0, d.step0);

    // point data of a chunk, loaded one chunk ahead of its generation: (Y, Z) of
    // the points wave + WV i that this wave generates, and weight component t % 4
    // of point t / 4 for t < 4 CHK
    constexpr int GPW = CHK / WV;  // points generated per wave
    static_assert(GPW * WV == CHK, "chunk and waves");
    const int wj = t >> 2, wc = t & 3;
    double nY[GPW], nZ[GPW], nW = 0.0;
    auto fetch = [&](int64_t j1) {
#pragma unroll
        for (int i = 0; i < GPW; ++i) {
            const int64_t j = j1 + wave + WV * i;
            nY[i] = j < jend ? pts[j].Y : 0.0;
            nZ[i] = j < jend ? pts[j].Z : 0.0;
        }
        nW = (wj < CHK && j1 + wj < jend) ? pts[j1 + wj].w[wc] : 0.0;
    };
    // twiddles of the fetched chunk into LDS buffer b (zeros past the end)
    auto generate = [&](int b) {
#pragma unroll
        for (int i = 0; i < GPW; ++i) {
            const int jj = wave + WV * i;
            const double2 tr = s_trig[lane];
            const double u = nY[i] * tr.x + nZ[i] * tr.y;
            const double2 step = twiddle(d.step0 * u);
            double2 sb = cmul(step, step);  // step^8: from one wave's rows to the next
            sb = cmul(sb, sb);
            sb = cmul(sb, sb);
            // start of the block exp(-i q(row0) u): with q rows from zero it is
            // step^row0 = (step^(8 WV))^blockIdx.y by binary powering (uniform over
            // the workgroup; the rounding of dq u is carried row0 times, a few
            // times the error of a sincos of q(row0) u, and each squaring adds one
            // rounding)
            double2 st;
            if (d.origin0 == 0.0) {
                double2 base = sb;
#pragma unroll
                for (int w = 1; w < WV; w += w) base = cmul(base, base);
                st = make_double2(1.0, 0.0);
                for (unsigned e = blockIdx.y; e != 0; e >>= 1) {
                    if (e & 1) st = cmul(st, base);
                    if (e > 1) base = cmul(base, base);
                }
            } else {
                st = twiddle(qrow0 * u);
            }
            s_step[b][jj][lane] = step;
            // wave starts st sb^w by the two-term recurrence in w (7 steps: the error
            // grows at most linearly in w)
            const double k8 = sb.x + sb.x;
            double2 pm = st, pc = cmul(st, sb);
            s_start[b][jj][0][lane] = pm;
            s_start[b][jj][1][lane] = pc;
#pragma unroll
            for (int w = 2; w < WV; ++w) {
                const double2 pn = make_double2(fma(k8, pc.x, -pm.x), fma(k8, pc.y, -pm.y));
                s_start[b][jj][w][lane] = pn;
                pm = pc;
                pc = pn;
            }
        }
        if (wj < CHK) s_w[b][wj][wc] = nW;
    };
    // sums of the nk points in buffer b; the operands of the next point are
    // requested before the current point is accumulated (as in the Cartesian loop)
    auto sum = [&](int b, int nk) {
        cart::Operands opa = polar_operands<WV, R>(s_start[b], s_step[b], s_w[b], 0, lane, wave);
        int jj = 0;
        for (; jj + 1 < nk; jj += 2) {
            const cart::Operands opb = polar_operands<WV, R>(s_start[b], s_step[b], s_w[b], jj + 1, lane, wave);
            __builtin_amdgcn_sched_barrier(0);
            polar_point<B, CH>(opa, acc);
            __builtin_amdgcn_sched_barrier(0);
            const int nxt = NB == 2 ? min(jj + 2, CHK - 1) : jj + 2;  // past the end: discarded
            opa = polar_operands<WV, R>(s_start[b], s_step[b], s_w[b], nxt, lane, wave);
            __builtin_amdgcn_sched_barrier(0);
            polar_point<B, CH>(opb, acc);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (jj < nk) polar_point<B, CH>(opa, acc);
    };

    fetch(jbeg);
    if (NB == 2) {
        // chunk c sits in buffer c & 1; chunk c + 1 is generated while chunk c is summed
        if (jbeg < jend) {
            generate(0);
            fetch(jbeg + CHK);
        }
        __syncthreads();
        int b = 0;
        for (int64_t j0 = jbeg; j0 < jend; j0 += CHK, b ^= 1) {
            if (j0 + CHK < jend) {
                generate(b ^ 1);  // its buffer was last read before the previous barrier
                fetch(j0 + 2 * CHK);
            }
            sum(b, (int)min((int64_t)CHK, jend - j0));
            __syncthreads();
        }
    } else {
        for (int64_t j0 = jbeg; j0 < jend; j0 += CHK) {
            if (j0 != jbeg) __syncthreads();  // the previous chunk's sums are done
            generate(0);
            fetch(j0 + CHK);  // arrives during the sums below
            __syncthreads();
            sum(0, (int)min((int64_t)CHK, jend - j0));
        }
    }
    const int64_t P = (int64_t)d.n0 * d.n1;
    double *dst = out + (int64_t)blockIdx.z * P * 8;
#pragma unroll
    for (int r = 0; r < B; ++r) {
        const int row = row0 + wave * B + r;
        if (row < d.n0 && gcol < d.n1) {
            double *o = dst + ((int64_t)row * d.n1 + gcol) * 8;
#pragma unroll
            for (int v = 0; v < 8; ++v) o[v] = cart::channel_value<CH>(acc[r], v);
        }
    }
}

// Waves per workgroup of the polar kernel: 8 (64 rows) unless the detector has
// at most 32 q rows.
static int polar_waves(const Detector &d) { return d.n0 > 4 * kPolarB ? 8 : 4; }

DirectPlan plan_direct_polar(const Detector &d, int64_t W, int64_t max_splits)
{
    DirectPlan p{};
    p.channels = 4;
    p.lanes = 64;
    const int rows = polar_waves(d) * kPolarB;
    p.col_blocks = (d.n1 + 63) / 64;
    p.row_blocks = (d.n0 + rows - 1) / rows;
    int64_t blocks = (int64_t)p.col_blocks * p.row_blocks;
    // half the Cartesian path's wave count: a polar workgroup holds its CU alone, and
    // two rounds of them over the chip measured faster than four (fewer partials too)
    int64_t want = (target_workgroups() * 2 / polar_waves(d) + blocks - 1) / blocks;
    int64_t max_split = (W + 8 * kPolarChunk - 1) / (8 * kPolarChunk);
    if (max_split < 1) max_split = 1;
    if (want > max_split) want = max_split;
    if (max_splits > 0 && want > max_splits) want = max_splits;
    if (want > 65535) want = 65535;
    if (want < 1) want = 1;
    int64_t per = (W + want - 1) / want;
    per = ((per + kPolarChunk - 1) / kPolarChunk) * kPolarChunk;
    if (per < kPolarChunk) per = kPolarChunk;
    p.per = per;
    p.nsplit = (int)((W + per - 1) / per);
    if (p.nsplit < 1) p.nsplit = 1;
    return p;
}

int launch_direct_polar(const PointRec *pts, int64_t W, const Detector &d, const DirectPlan &p,
                        double *partial, hipStream_t s, int n_rot)
{
    if ((int64_t)p.nsplit * n_rot > 65535) return NUMAG_E_INVALID;
    dim3 grid(p.col_blocks, p.row_blocks, p.nsplit * n_rot);
    TimedLaunch timed(NUMAG_KERNEL_DIRECT, s);
#define NUMAG_LAUNCH_POLAR(WV, CH)                                                                          \
    hipLaunchKernelGGL((direct_polar_kernel<WV, CH>), grid, dim3(64 * WV), 0, s, pts, W, p.per, p.nsplit, d, \
                       partial)
#define NUMAG_LAUNCH_POLAR_CH(WV)                  \
    switch (p.channels) {                          \
        case 1: NUMAG_LAUNCH_POLAR(WV, 1); break;  \
        case 3: NUMAG_LAUNCH_POLAR(WV, 3); break;  \
        default: NUMAG_LAUNCH_POLAR(WV, 4); break; \
    }
    if (polar_waves(d) == 8) {
        NUMAG_LAUNCH_POLAR_CH(8);
    } else {
        NUMAG_LAUNCH_POLAR_CH(4);
    }
#undef NUMAG_LAUNCH_POLAR_CH
#undef NUMAG_LAUNCH_POLAR
    NUMAG_HIP_CHECK(hipGetLastError());
    return NUMAG_OK;
}

// Dilute orientational average on a polar detector, one object and a group of nr
// rotations: F_r(p) = sum of the nsp split partials of rotation r (part[r nsp + s]
// over the Ph pixels summed), and spec[p] += scale sum_r F_r(p) F_r(p)^H in
// rotation order.  nh > 0: the partials cover the theta columns [0, nh) of a
// detector with 2 nh columns, and column m + nh receives conj G (real weights).
__global__ void spectral_rotations_kernel(const double *__restrict__ part, int nr, int nsp, int64_t Ph, int n1,
                                          int nh, double scale, double *__restrict__ spec)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= Ph) return;
    double g[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) g[v] = 0.0;
    for (int r = 0; r < nr; ++r) {
        double F[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) F[v] = 0.0;
        for (int sp = 0; sp < nsp; ++sp) {
            const double *src = part + ((int64_t)(r * nsp + sp) * Ph + p) * 8;
#pragma unroll
            for (int v = 0; v < 8; ++v) F[v] += src[v];
        }
        // G_ab += F_a conj(F_b): diagonal, then the upper triangle
#pragma unroll
        for (int a = 0; a < 4; ++a) g[a] += F[2 * a] * F[2 * a] + F[2 * a + 1] * F[2 * a + 1];
        const int pa[6] = {0, 0, 0, 1, 1, 2};
        const int pb[6] = {1, 2, 3, 2, 3, 3};
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            const double ar = F[2 * pa[t]], ai = F[2 * pa[t] + 1];
            const double br = F[2 * pb[t]], bi = F[2 * pb[t] + 1];
            g[4 + 2 * t] += ar * br + ai * bi;
            g[5 + 2 * t] += ai * br - ar * bi;
        }
    }
    const int64_t pf = nh > 0 ? (p / nh) * n1 + p % nh : p;
    double *o = spec + pf * 16;
#pragma unroll
    for (int v = 0; v < 16; ++v) o[v] += scale * g[v];
    if (nh > 0) {
        double *m = spec + (pf + nh) * 16;
#pragma unroll
        for (int v = 0; v < 16; ++v) m[v] += (v >= 5 && (v & 1)) ? -scale * g[v] : scale * g[v];
    }
}

int launch_spectral_rotations(const double *part, int nr, int nsp, int64_t Ph, int n1, int nh, double scale,
                              double *spec, hipStream_t s)
{
    if (Ph <= 0 || nr <= 0) return NUMAG_OK;
    hipLaunchKernelGGL(spectral_rotations_kernel, dim3((unsigned)((Ph + 255) / 256)), dim3(256), 0, s, part, nr, nsp,
                       Ph, n1, nh, scale, spec);
    NUMAG_HIP_CHECK(hipGetLastError());
    return NUMAG_OK;
}

}  // namespace numag
