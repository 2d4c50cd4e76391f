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
// so the per-(point, column) generation (u, two sincos for the step and the
// block start exp(-i q(row0) u), the wave starts by powers of step^8) is shared
// by 8 WV rows.
// ---------------------------------------------------------------------------
constexpr int kPolarChunk = 8;
constexpr int kPolarB = 8;

// Operands of point jj for this lane: ez = the wave's start phasor, dz = the q step.
template <int WV>
__device__ __forceinline__ cart::Operands polar_operands(const double2 (&s_start)[kPolarChunk + 1][WV][64],
                                                         const double2 (&s_step)[kPolarChunk + 1][64],
                                                         const double (&s_k)[kPolarChunk + 1][64],
                                                         const double (&s_w)[kPolarChunk + 1][4], int jj, int lane,
                                                         int wave)
{
    cart::Operands o;
    o.ez = s_start[jj][wave][lane];
    o.dz = s_step[jj][lane];
    o.k = s_k[jj][lane];
#pragma unroll
    for (int v = 0; v < 4; ++v) o.w[v] = s_w[jj][v];
    return o;
}

// Adds one point to the lane's B q rows: start, one step, then the recurrence.
template <int B, int CH>
__device__ __forceinline__ void polar_point(const cart::Operands &o, double (&acc)[B][2 * CH])
{
    double2 pm = o.ez;
    double2 pc = cmul(pm, o.dz);
    cart::add_weighted<CH>(o, pm, acc[0]);
    cart::add_weighted<CH>(o, pc, acc[1]);
#pragma unroll
    for (int r = 2; r < B; ++r) {
        const double2 pn = make_double2(fma(o.k, pc.x, -pm.x), fma(o.k, pc.y, -pm.y));
        cart::add_weighted<CH>(o, pn, acc[r]);
        pm = pc;
        pc = pn;
    }
}

template <int WV, int CH>
__global__ __launch_bounds__(64 * WV, 8 / WV) void direct_polar_kernel(const PointRec *__restrict__ pts, int64_t W,
                                                                      int64_t per, Detector d,
                                                                      double *__restrict__ out)
{
    constexpr int B = kPolarB;
    constexpr int ROWS = WV * B;
    // one row per point of a chunk plus one the pipelined loop may read past the end
    __shared__ double2 s_start[kPolarChunk + 1][WV][64];
    __shared__ double2 s_step[kPolarChunk + 1][64];
    __shared__ double s_k[kPolarChunk + 1][64];
    __shared__ double s_w[kPolarChunk + 1][4];
    __shared__ double2 s_trig[64];  // (sin, cos) of the lane's column angle

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int col0 = blockIdx.x * 64;
    const int row0 = blockIdx.y * ROWS;
    const int64_t jbeg = (int64_t)blockIdx.z * per;
    const int64_t jend = min(W, jbeg + per);

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
    }  // published by the first barrier of the chunk loop
    const double qrow0 = axis_value(d.origin0, row0, d.step0);

    // point data of a chunk, loaded one chunk ahead: (Y, Z) of the points
    // wave + WV i that this wave generates, and weight component t % 4 of point
    // t / 4 for t < 4 kPolarChunk
    constexpr int GPW = kPolarChunk / WV;  // points generated per wave
    static_assert(GPW * WV == kPolarChunk, "chunk and waves");
    const int wj = t >> 2, wc = t & 3;
    double nY[GPW], nZ[GPW], nW = 0.0;
#pragma unroll
    for (int i = 0; i < GPW; ++i) {
        const int64_t j = jbeg + wave + WV * i;
        nY[i] = j < jend ? pts[j].Y : 0.0;
        nZ[i] = j < jend ? pts[j].Z : 0.0;
    }
    if (wj < kPolarChunk && jbeg + wj < jend) nW = pts[jbeg + wj].w[wc];

    for (int64_t j0 = jbeg; j0 < jend; j0 += kPolarChunk) {
        const int nk = (int)min((int64_t)kPolarChunk, jend - j0);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < GPW; ++i) {
            const int jj = wave + WV * i;
            const double Y = nY[i], Z = nZ[i];  // zero past the end
            const double2 tr = s_trig[lane];
            const double u = Y * tr.x + Z * tr.y;
            const double2 step = twiddle(d.step0 * u);
            double2 sb = cmul(step, step);  // step^8: from one wave's rows to the next
            sb = cmul(sb, sb);
            sb = cmul(sb, sb);
            double2 st = twiddle(qrow0 * u);  // start of the block
            s_step[jj][lane] = step;
            s_k[jj][lane] = step.x + step.x;
#pragma unroll
            for (int w = 0; w < WV; ++w) {
                s_start[jj][w][lane] = st;
                st = cmul(st, sb);
            }
        }
        if (wj < kPolarChunk) s_w[wj][wc] = nW;  // zero past the end
        // request the next chunk's point data; it arrives during the sums below
        const int64_t j1 = j0 + kPolarChunk;
#pragma unroll
        for (int i = 0; i < GPW; ++i) {
            const int64_t j = j1 + wave + WV * i;
            nY[i] = j < jend ? pts[j].Y : 0.0;
            nZ[i] = j < jend ? pts[j].Z : 0.0;
        }
        nW = (wj < kPolarChunk && j1 + wj < jend) ? pts[j1 + wj].w[wc] : 0.0;
        __syncthreads();
        // operands of the next point are requested before the current point is
        // accumulated (as in the Cartesian loop)
        cart::Operands opa = polar_operands<WV>(s_start, s_step, s_k, s_w, 0, lane, wave);
        int jj = 0;
        for (; jj + 1 < nk; jj += 2) {
            const cart::Operands opb = polar_operands<WV>(s_start, s_step, s_k, s_w, jj + 1, lane, wave);
            __builtin_amdgcn_sched_barrier(0);
            polar_point<B, CH>(opa, acc);
            __builtin_amdgcn_sched_barrier(0);
            opa = polar_operands<WV>(s_start, s_step, s_k, s_w, jj + 2, lane, wave);  // row kPolarChunk at most
            __builtin_amdgcn_sched_barrier(0);
            polar_point<B, CH>(opb, acc);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (jj < nk) polar_point<B, CH>(opa, acc);
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

DirectPlan plan_direct_polar(const Detector &d, int64_t W)
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
                        double *partial, hipStream_t s)
{
    dim3 grid(p.col_blocks, p.row_blocks, p.nsplit);
    TimedLaunch timed(NUMAG_KERNEL_DIRECT, s);
#define NUMAG_LAUNCH_POLAR(WV, CH) \
    hipLaunchKernelGGL((direct_polar_kernel<WV, CH>), grid, dim3(64 * WV), 0, s, pts, W, p.per, d, partial)
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

}  // namespace numag
