// Direct Fourier sums on the paper's polar (q, theta) detector (Sec. 3.2):
// S_c(q_i, theta_m) = sum_j w_{j,c} exp(-i q_i u_m(j)),  u_m = Y sin(theta_m) + Z cos(theta_m).
#include "cartesian_sum.h"

namespace numag {


// ---------------------------------------------------------------------------
// Polar direct sum.  The phase q_i u_m with u_m = Y sin(theta_m) + Z cos(theta_m)
// does not separate, but along q it is a geometric sequence: a lane owns one theta
// column and walks 8 q rows, the first from its row group's start phasor, the
// second by one step exp(-i dq u), the rest by the two-term recurrence
// p_{r+1} = 2 cos(dq u) p_r - p_{r-1}.
//
// Workgroup shapes (PolarShape): WV waves, CW theta columns; a wave covers its CW
// columns with 64 / CW row groups of 8 rows, so the workgroup covers
// ROWS = 8 WV 64 / CW q rows.  The per-(point, column) generation -- u, one sincos
// for the step, the block start exp(-i q(row0) u) as a power of the step, the row
// groups' starts by the same recurrence in step^8 -- is done once per workgroup
// and shared by its ROWS rows: narrower column blocks share it over more rows (and
// do fewer generations per workgroup) at the price of padding on detectors with
// fewer rows.
// ---------------------------------------------------------------------------
constexpr int kPolarB = 8;  // q rows per lane

// The workgroup shapes the launcher instantiates (index = DirectPlan::shape).
struct PolarShapeDesc {
    int waves, cols, chunk, buffers;
};
constexpr PolarShapeDesc kPolarShapes[kPolarShapeCount] = {
    {8, 64, 8, 2},   // 0: 64 rows x 64 columns, double-buffered chunks of 8 points
    {4, 64, 8, 1},   // 1: 32 rows x 64 columns (detectors of at most 32 q rows), two per CU
    {8, 32, 8, 2},   // 2: 128 rows x 32 columns, double-buffered
    {8, 16, 16, 1},  // 3: 256 rows x 16 columns, single-buffered chunks of 16 points
    {8, 16, 8, 2},   // 4: 256 rows x 16 columns, double-buffered chunks of 8 points
};

int polar_shape_rows(int shape)
{
    const PolarShapeDesc &s = kPolarShapes[shape];
    return kPolarB * s.waves * (64 / s.cols);
}
int polar_shape_cols(int shape) { return kPolarShapes[shape].cols; }
int polar_shape_waves(int shape) { return kPolarShapes[shape].waves; }

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

// grid.z = rotation r of a group x split sp (nsp splits per rotation); the points of
// rotation r are pts[r wrot, (r + 1) wrot).  One rotation: wrot = W, nsp = grid.z.
template <int WV, int CW, int CHK, int NB, int CH>
__global__ __launch_bounds__(64 * WV, 8 / WV) void direct_polar_kernel(const PointRec *__restrict__ pts,
                                                                      int64_t wrot, int64_t per, int nsp, Detector d,
                                                                      double *__restrict__ out)
{
    constexpr int B = kPolarB;
    constexpr int NT = 64 * WV;        // threads
    constexpr int LPC = 64 / CW;       // row groups per wave
    constexpr int G = WV * LPC;        // row groups per workgroup
    constexpr int ROWS = B * G;
    constexpr int GEN = CHK * CW;      // (point, column) generations per chunk
    constexpr int GPT = (GEN + NT - 1) / NT;  // generations per thread
    static_assert(CW == 64 || CW == 32 || CW == 16, "columns per workgroup");
    static_assert(GEN % 64 == 0, "generation is wave-uniform");
    static_assert(4 * CHK <= NT, "one weight component per thread");
    // one row per point of a chunk; single-buffered, plus one the pipelined loop
    // may read past the end (double-buffered, that read is clamped instead)
    constexpr int R = NB == 2 ? CHK : CHK + 1;
    __shared__ double2 s_start[NB][R][G][CW];  // start phasor of each row group and column
    __shared__ double2 s_step[NB][R][CW];      // q step of each column
    __shared__ double s_w[NB][R][4];
    __shared__ double2 s_trig[CW];             // (sin, cos) of the column angles

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int col0 = blockIdx.x * CW;
    const int row0 = blockIdx.y * ROWS;
    const int64_t rbase = (int64_t)(blockIdx.z / nsp) * wrot;
    const int64_t jbeg = rbase + (int64_t)(blockIdx.z % nsp) * per;
    const int64_t jend = min(rbase + wrot, jbeg + per);

    double acc[B][2 * CH];
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
        for (int v = 0; v < 2 * CH; ++v) acc[r][v] = 0.0;

    if (t < CW) {
        const double theta = (2.0 * 3.141592653589793 * (double)(col0 + t)) / (double)d.n_theta;
        double sth, cth;
        sincos(theta, &sth, &cth);
        s_trig[t] = make_double2(sth, cth);
    }
    __syncthreads();
    const double qrow0 = axis_value(d.origin0, row0, d.step0);

    // generation e = t + NT i of a chunk (e < GEN): point e / CW, column e % CW.
    // Point data of a chunk is loaded one chunk ahead of its generation: (Y, Z) of
    // the thread's generation points, and weight component t % 4 of point t / 4
    // for t < 4 CHK.
    const int wj = t >> 2, wc = t & 3;
    double nY[GPT], nZ[GPT], nW = 0.0;
    auto fetch = [&](int64_t j1) {
#pragma unroll
        for (int i = 0; i < GPT; ++i) {
            const int e = t + NT * i;
            const int64_t j = j1 + e / CW;
            const bool ok = e < GEN && j < jend;
            nY[i] = ok ? pts[j].Y : 0.0;
            nZ[i] = ok ? pts[j].Z : 0.0;
        }
        nW = (wj < CHK && j1 + wj < jend) ? pts[j1 + wj].w[wc] : 0.0;
    };
    // twiddles of the fetched chunk into LDS buffer b (zeros past the end)
    auto generate = [&](int b) {
#pragma unroll
        for (int i = 0; i < GPT; ++i) {
            const int e = t + NT * i;
            if (e >= GEN) break;  // wave-uniform
            const int jj = e / CW, c = e % CW;
            const double2 tr = s_trig[c];
            const double u = nY[i] * tr.x + nZ[i] * tr.y;
            const double2 step = twiddle(d.step0 * u);
            double2 sb = cmul(step, step);  // step^8: from one row group to the next
            sb = cmul(sb, sb);
            sb = cmul(sb, sb);
            // start of the block exp(-i q(row0) u): with q rows from zero it is
            // step^row0 = (step^ROWS)^blockIdx.y by binary powering (uniform over
            // the workgroup; the rounding of dq u is carried row0 times, a few
            // times the error of a sincos of q(row0) u, and each squaring adds one
            // rounding)
            double2 st;
            if (d.origin0 == 0.0) {
                double2 base = sb;
#pragma unroll
                for (int g = 1; g < G; g += g) base = cmul(base, base);
                st = make_double2(1.0, 0.0);
                for (unsigned ex = blockIdx.y; ex != 0; ex >>= 1) {
                    if (ex & 1) st = cmul(st, base);
                    if (ex > 1) base = cmul(base, base);
                }
            } else {
                st = twiddle(qrow0 * u);
            }
            s_step[b][jj][c] = step;
            // row-group starts st sb^g by the two-term recurrence in g (G - 1 steps:
            // the error grows at most linearly in g)
            const double k8 = sb.x + sb.x;
            double2 pm = st, pc = cmul(st, sb);
            s_start[b][jj][0][c] = pm;
            s_start[b][jj][1][c] = pc;
#pragma unroll
            for (int g = 2; g < G; ++g) {
                const double2 pn = make_double2(fma(k8, pc.x, -pm.x), fma(k8, pc.y, -pm.y));
                s_start[b][jj][g][c] = pn;
                pm = pc;
                pc = pn;
            }
        }
        if (wj < CHK) s_w[b][wj][wc] = nW;
    };
    // this lane's column and row group
    const int lc = lane % CW;
    const int lg = wave * LPC + lane / CW;
    auto operands = [&](int b, int jj) {
        cart::Operands o;
        o.ez = s_start[b][jj][lg][lc];
        o.dz = s_step[b][jj][lc];
        o.k = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) o.w[v] = s_w[b][jj][v];
        return o;
    };
    // sums of the nk points in buffer b; the operands of the next point are
    // requested before the current point is accumulated (as in the Cartesian loop)
    auto sum = [&](int b, int nk) {
        cart::Operands opa = operands(b, 0);
        int jj = 0;
        for (; jj + 1 < nk; jj += 2) {
            const cart::Operands opb = operands(b, jj + 1);
            __builtin_amdgcn_sched_barrier(0);
            polar_point<B, CH>(opa, acc);
            __builtin_amdgcn_sched_barrier(0);
            const int nxt = NB == 2 ? min(jj + 2, CHK - 1) : jj + 2;  // past the end: discarded
            opa = operands(b, nxt);
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
    const int gcol = col0 + lc;
#pragma unroll
    for (int r = 0; r < B; ++r) {
        const int row = row0 + lg * B + r;
        if (row < d.n0 && gcol < d.n1) {
            double *o = dst + ((int64_t)row * d.n1 + gcol) * 8;
#pragma unroll
            for (int v = 0; v < 8; ++v) o[v] = cart::channel_value<CH>(acc[r], v);
        }
    }
}

// Default workgroup shape: 32 rows on detectors of at most 32 q rows; otherwise,
// among the double-buffered shapes, the one with the fewest estimated VALU
// instructions per (point, theta column): the sums (about 10.3 per term over the
// padded rows) plus one generation per row block (about 150 for the sincos,
// powers and stores, plus 2 per row group).  Measured on 262,144 points: 256 x 256
// and 1000 x 1000 detectors take shape 4 (0.72 and 0.68 of the FP64 peak, against
// 0.59 and 0.57 for shape 0), 128 x 128 takes shape 2 (0.68 against 0.63).
int default_polar_shape(const Detector &d)
{
    if (d.n0 <= 32) return 1;
    int best = 0;
    double best_cost = 0.0;
    for (int sh : {0, 2, 4}) {
        const int rows = polar_shape_rows(sh), cols = polar_shape_cols(sh);
        const double rb = (double)((d.n0 + rows - 1) / rows);
        const double cpad = (double)(((d.n1 + cols - 1) / cols) * cols) / (double)d.n1;
        const double cost = cpad * rb * (10.3 * rows + 150.0 + 2.0 * rows / kPolarB);
        if (sh == 0 || cost < best_cost) {
            best = sh;
            best_cost = cost;
        }
    }
    return best;
}

DirectPlan plan_direct_polar(const Detector &d, int64_t W, int64_t max_splits, int shape, int target_wgs)
{
    DirectPlan p{};
    p.channels = 4;
    const TuneShape ts = current_tune_shape(kTuneDirect, d, W);
    p.shape = shape >= 0 && shape < kPolarShapeCount ? shape : ts.shape;
    if (d.n0 > 32 && p.shape == 1) p.shape = 0;  // the 4-wave shape serves short detectors only
    const PolarShapeDesc &sd = kPolarShapes[p.shape];
    p.lanes = sd.cols;
    const int rows = polar_shape_rows(p.shape);
    p.col_blocks = (d.n1 + sd.cols - 1) / sd.cols;
    p.row_blocks = (d.n0 + rows - 1) / rows;
    int64_t blocks = (int64_t)p.col_blocks * p.row_blocks;
    const int tw = target_wgs > 0 ? target_wgs : ts.target;
    int64_t want = (tw + blocks - 1) / blocks;
    int64_t max_split = (W + 8 * sd.chunk - 1) / (8 * sd.chunk);
    if (max_split < 1) max_split = 1;
    if (want > max_split) want = max_split;
    if (max_splits > 0 && want > max_splits) want = max_splits;
    if (want > 65535) want = 65535;
    if (want < 1) want = 1;
    int64_t per = (W + want - 1) / want;
    per = ((per + sd.chunk - 1) / sd.chunk) * sd.chunk;
    if (per < sd.chunk) per = sd.chunk;
    p.per = per;
    p.nsplit = (int)((W + per - 1) / per);
    if (p.nsplit < 1) p.nsplit = 1;
    return p;
}

int launch_direct_polar(const PointRec *pts, int64_t W, const Detector &d, const DirectPlan &p,
                        double *partial, hipStream_t s, int n_rot)
{
    if ((int64_t)p.nsplit * n_rot > 65535) return NUMAG_E_INVALID;
    if (p.shape < 0 || p.shape >= kPolarShapeCount) return NUMAG_E_INVALID;
    const PolarShapeDesc &sd = kPolarShapes[p.shape];
    dim3 grid(p.col_blocks, p.row_blocks, p.nsplit * n_rot);
    TimedLaunch timed(NUMAG_KERNEL_DIRECT, s);
#define NUMAG_LAUNCH_POLAR(WV, CW, CHK, NB, CH)                                                                   \
    hipLaunchKernelGGL((direct_polar_kernel<WV, CW, CHK, NB, CH>), grid, dim3(64 * WV), 0, s, pts, W, p.per, \
                       p.nsplit, d, partial)
#define NUMAG_LAUNCH_POLAR_CH(WV, CW, CHK, NB)                  \
    switch (p.channels) {                                       \
        case 1: NUMAG_LAUNCH_POLAR(WV, CW, CHK, NB, 1); break;  \
        case 3: NUMAG_LAUNCH_POLAR(WV, CW, CHK, NB, 3); break;  \
        default: NUMAG_LAUNCH_POLAR(WV, CW, CHK, NB, 4); break; \
    }
    switch (p.shape) {
        case 0: NUMAG_LAUNCH_POLAR_CH(8, 64, 8, 2); break;
        case 1: NUMAG_LAUNCH_POLAR_CH(4, 64, 8, 1); break;
        case 2: NUMAG_LAUNCH_POLAR_CH(8, 32, 8, 2); break;
        case 3: NUMAG_LAUNCH_POLAR_CH(8, 16, 16, 1); break;
        default: NUMAG_LAUNCH_POLAR_CH(8, 16, 8, 2); break;
    }
#undef NUMAG_LAUNCH_POLAR_CH
#undef NUMAG_LAUNCH_POLAR
    (void)sd;
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
