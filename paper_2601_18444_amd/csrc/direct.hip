// Direct Fourier sums on gfx950: the general (any point cloud, any rotation) path.
//
// Sums (Sec. 3.3, DSFT):  S_c(q_p) = sum_j w_{j,c} exp(-i q_p . X_j),  q = (0, q_y, q_z).
//
// Cartesian detector.  The phase separates in the lab frame,
//   exp(-i (q_y Y + q_z Z)) = exp(-i q_y Y) * exp(-i q_z Z),
// so a term costs one complex multiply for its phasor plus eight FMAs for the
// four complex channel sums; there is no transcendental per term.  A wave owns
// A detector rows x (64 lanes * B columns); per point a lane takes its row
// twiddle exp(-i q_y Y) (wave-uniform, from LDS), its first-column twiddle
// exp(-i q_z(k_lane) Z) (from LDS) and walks its B columns with the
// column-step twiddle exp(-i dq_z Z).  Twiddles are generated per chunk of
// points by the whole workgroup in FP64 (sincos plus short recurrences), and
// everything is accumulated in FP64: on gfx950 an FP64 FMA issues at the same
// rate as an unpacked FP32 FMA, so FP64 costs no throughput here and removes
// the FP32 phase/accumulation error budget entirely.
//
// Polar detector (the paper's (q, theta) grid).  The phase q u_m(j) with
// u_m = Y sin(theta_m) + Z cos(theta_m) is not separable; lanes own theta
// columns and walk B consecutive q rows with the step twiddle exp(-i dq u).
//
// Work is split over point ranges (split-K); a fixed-order FP64 combine sums
// the partial results, so results are bitwise reproducible.
#include "cartesian_sum.h"

namespace numag {

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// exp(-i phi) = (cos phi, -sin phi)
__device__ __forceinline__ double2 twiddle(double phi)
{
    double s, c;
    sincos(phi, &s, &c);
    return make_double2(c, -s);
}

// Detector axis value origin + i * step, as one rounded product and one rounded
// sum (the detector definition; must not be fused).
__device__ __forceinline__ double axis_value(double origin, int i, double step)
{
#pragma clang fp contract(off)
    double t = (double)i * step;
    return origin + t;
}

Detector make_detector(const numag_qgrid &g)
{
    Detector d{};
    d.kind = g.kind;
    d.n0 = g.n0;
    d.n1 = g.n1;
    d.qmax = g.qmax;
    if (g.kind == NUMAG_GRID_CARTESIAN) {
        d.step0 = g.n0 > 1 ? (2.0 * g.qmax) / (double)(g.n0 - 1) : 0.0;
        d.step1 = g.n1 > 1 ? (2.0 * g.qmax) / (double)(g.n1 - 1) : 0.0;
        d.origin0 = g.n0 > 1 ? -g.qmax : 0.0;
        d.origin1 = g.n1 > 1 ? -g.qmax : 0.0;
    } else {
        d.step0 = g.n0 > 1 ? g.qmax / (double)(g.n0 - 1) : 0.0;
        d.step1 = 0.0;  // theta_m = (2 pi m) / n_theta, computed as written
        d.origin0 = 0.0;
        d.origin1 = 0.0;
    }
    return d;
}

// ---------------------------------------------------------------------------
// sample assembly and rotation (Sec. 3.2): X = R (x + r^k), w' = (n, R m).
// ---------------------------------------------------------------------------
__global__ void prepare_points_kernel(const double *__restrict__ pos, const double *__restrict__ nuc,
                                      const double *__restrict__ mag, int64_t W, int reg,
                                      numag_regular g, const int64_t *__restrict__ off, int64_t K,
                                      const double *__restrict__ obj_pos, Rot R,
                                      PointRec *__restrict__ out)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= W) return;
    double x[3];
    if (reg) {
        int64_t nyz = (int64_t)g.n[1] * g.n[2];
        int64_t ix = j / nyz, rem = j % nyz;
        int64_t iy = rem / g.n[2], iz = rem % g.n[2];
        x[0] = g.origin[0] + (double)ix * g.step[0];
        x[1] = g.origin[1] + (double)iy * g.step[1];
        x[2] = g.origin[2] + (double)iz * g.step[2];
    } else {
        x[0] = pos[3 * j + 0];
        x[1] = pos[3 * j + 1];
        x[2] = pos[3 * j + 2];
    }
    if (obj_pos != nullptr) {
        int64_t k = 0;
        if (K > 1 && off != nullptr) {
            int64_t lo = 0, hi = K - 1;  // largest k with off[k] <= j
            while (lo < hi) {
                int64_t mid = (lo + hi + 1) >> 1;
                if (off[mid] <= j) lo = mid; else hi = mid - 1;
            }
            k = lo;
        }
        x[0] += obj_pos[3 * k + 0];
        x[1] += obj_pos[3 * k + 1];
        x[2] += obj_pos[3 * k + 2];
    }
    PointRec r;
    r.Y = R.m[3] * x[0] + R.m[4] * x[1] + R.m[5] * x[2];
    r.Z = R.m[6] * x[0] + R.m[7] * x[1] + R.m[8] * x[2];
    r.w[0] = nuc != nullptr ? nuc[j] : 0.0;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0;
    if (mag != nullptr) {
        m0 = mag[3 * j + 0];
        m1 = mag[3 * j + 1];
        m2 = mag[3 * j + 2];
    }
    r.w[1] = R.m[0] * m0 + R.m[1] * m1 + R.m[2] * m2;
    r.w[2] = R.m[3] * m0 + R.m[4] * m1 + R.m[5] * m2;
    r.w[3] = R.m[6] * m0 + R.m[7] * m1 + R.m[8] * m2;
    r.pad[0] = r.pad[1] = 0.0;
    out[j] = r;
}

int launch_prepare_points(const double *pos, const double *nuc, const double *mag, int64_t W,
                          const numag_regular *regular, const int64_t *d_offsets, int64_t K,
                          const double *obj_pos, const Rot &R, PointRec *out, hipStream_t s)
{
    if (W <= 0) return NUMAG_OK;
    numag_regular g{};
    if (regular != nullptr) g = *regular;
    const int tpb = 256;
    int64_t blocks = (W + tpb - 1) / tpb;
    hipLaunchKernelGGL(prepare_points_kernel, dim3((unsigned)blocks), dim3(tpb), 0, s, pos, nuc, mag, W,
                       regular != nullptr ? 1 : 0, g, d_offsets, K, obj_pos, R, out);
    NUMAG_HIP_CHECK(hipGetLastError());
    return NUMAG_OK;
}

// ---------------------------------------------------------------------------
// Cartesian direct sum.
// ---------------------------------------------------------------------------
constexpr int kWaves = cart::kWaves;
constexpr int kThreads = cart::kThreads;
constexpr int kChunk = cart::kChunk;

struct PrepLoader {
    const PointRec *__restrict__ pts;
    __device__ __forceinline__ cart::PointPart load(int64_t j, int slot) const
    {
        const PointRec &r = pts[j];
        return cart::PointPart{r.Y, r.Z, slot < 4 ? r.w[slot] : 0.0};
    }
};

template <int LR>
__global__ __launch_bounds__(kThreads, 2) void direct_cartesian_kernel(
    const PointRec *__restrict__ pts, int64_t W, int64_t per, Detector d, double *__restrict__ out)
{
    using T = cart::Tile<LR>;
    __shared__ cart::Smem<LR> sm;
    const int col0 = blockIdx.x * T::COLS;
    const int row0 = blockIdx.y * T::ROWS;
    const int64_t jbeg = (int64_t)blockIdx.z * per;
    const int64_t jend = min(W, jbeg + per);
    double acc[cart::kB][8];
    cart::zero(acc);
    cart::accumulate<LR>(PrepLoader{pts}, jbeg, jend, d, col0, row0, sm, acc);

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t P = (int64_t)d.n0 * d.n1;
    double *dst = out + (int64_t)blockIdx.z * P * 8;
    const int row = T::row(row0, lane, wave);
    if (row >= d.n0) return;
#pragma unroll
    for (int c = 0; c < cart::kB; ++c) {
        const int col = T::col(col0, lane, c);
        if (col < d.n1) {
            double *o = dst + ((int64_t)row * d.n1 + col) * 8;
#pragma unroll
            for (int v = 0; v < 8; ++v) o[v] = acc[c][v];
        }
    }
}

static int target_workgroups()
{
    static int cached = -1;
    if (cached < 0) {
        const char *e = getenv("NUMAG_TARGET_WGS");
        cached = e != nullptr ? atoi(e) : 0;
        if (cached <= 0) cached = 2048;
    }
    return cached;
}

DirectPlan plan_direct_cartesian(const Detector &d, int64_t W)
{
    DirectPlan p{};
    p.lanes = cart::choose_lanes(d.n1);
    const int cols = p.lanes * cart::kB, rows = kThreads / p.lanes;
    p.col_blocks = (d.n1 + cols - 1) / cols;
    p.row_blocks = (d.n0 + rows - 1) / rows;
    int64_t blocks = (int64_t)p.col_blocks * p.row_blocks;
    int64_t want = (target_workgroups() + blocks - 1) / blocks;
    // each split should own a few chunks
    int64_t max_split = (W + 4 * kChunk - 1) / (4 * kChunk);
    if (max_split < 1) max_split = 1;
    if (want > max_split) want = max_split;
    if (want > 65535) want = 65535;
    if (want < 1) want = 1;
    int64_t per = (W + want - 1) / want;
    per = ((per + kChunk - 1) / kChunk) * kChunk;
    if (per < kChunk) per = kChunk;
    p.per = per;
    p.nsplit = (int)((W + per - 1) / per);
    if (p.nsplit < 1) p.nsplit = 1;
    return p;
}

size_t direct_partial_bytes(const DirectPlan &p, const Detector &d)
{
    return (size_t)p.nsplit * (size_t)d.n0 * (size_t)d.n1 * 8 * sizeof(double);
}

int launch_direct_cartesian(const PointRec *pts, int64_t W, const Detector &d, const DirectPlan &p,
                            double *partial, hipStream_t s)
{
    dim3 grid(p.col_blocks, p.row_blocks, p.nsplit);
    dim3 block(kThreads);
    TimedLaunch timed(NUMAG_KERNEL_DIRECT, s);
#define NUMAG_LAUNCH_CART(LR) \
    hipLaunchKernelGGL((direct_cartesian_kernel<LR>), grid, block, 0, s, pts, W, p.per, d, partial)
    switch (p.lanes) {
        case 8: NUMAG_LAUNCH_CART(8); break;
        case 16: NUMAG_LAUNCH_CART(16); break;
        case 32: NUMAG_LAUNCH_CART(32); break;
        default: NUMAG_LAUNCH_CART(64); break;
    }
#undef NUMAG_LAUNCH_CART
    NUMAG_HIP_CHECK(hipGetLastError());
    return NUMAG_OK;
}

// ---------------------------------------------------------------------------
// Polar direct sum.  The phase q_i u_m with u_m = Y sin(theta_m) + Z cos(theta_m)
// does not separate, but along q it is a geometric sequence: lanes own theta
// columns and each walks 8 q rows, the first by the row-group start, the second
// by one step exp(-i dq u), the rest by the two-term recurrence
// p_{r+1} = 2 cos(dq u) p_r - p_{r-1}.  A workgroup of WV waves covers 8 WV rows,
// so the per-(point, column) generation (u, one sincos for the step, the block
// start step^row0 by squaring, the wave starts by powers of step^8) is shared
// by 8 WV rows.
// ---------------------------------------------------------------------------
constexpr int kPolarChunk = 8;
constexpr int kPolarB = 8;

// z^e for e >= 0 by binary powering (|z| = 1; relative error about e ulp).
__device__ __forceinline__ double2 cpow_int(double2 z, int e)
{
    double2 r = make_double2(1.0, 0.0);
    while (e > 0) {
        if (e & 1) r = cart::cmul(r, z);
        z = cart::cmul(z, z);
        e >>= 1;
    }
    return r;
}

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
template <int B>
__device__ __forceinline__ void polar_point(const cart::Operands &o, double (&acc)[B][8])
{
    double2 pm = o.ez;
    double2 pc = cart::cmul(pm, o.dz);
    cart::add_weighted(o, pm, acc[0]);
    cart::add_weighted(o, pc, acc[1]);
#pragma unroll
    for (int r = 2; r < B; ++r) {
        const double2 pn = make_double2(fma(o.k, pc.x, -pm.x), fma(o.k, pc.y, -pm.y));
        cart::add_weighted(o, pn, acc[r]);
        pm = pc;
        pc = pn;
    }
}

template <int WV>
__global__ __launch_bounds__(64 * WV, 8 / WV) void direct_polar_kernel(const PointRec *__restrict__ pts, int64_t W,
                                                                      int64_t per, Detector d,
                                                                      double *__restrict__ out)
{
    constexpr int B = kPolarB;
    constexpr int ROWS = WV * B;
    static_assert(kPolarChunk % WV == 0 || WV % kPolarChunk == 0, "chunk and waves");
    // one row per point of a chunk plus one the pipelined loop may read past the end
    __shared__ double2 s_start[kPolarChunk + 1][WV][64];
    __shared__ double2 s_step[kPolarChunk + 1][64];
    __shared__ double s_k[kPolarChunk + 1][64];
    __shared__ double s_w[kPolarChunk + 1][4];

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int col0 = blockIdx.x * 64;
    const int row0 = blockIdx.y * ROWS;
    const int64_t jbeg = (int64_t)blockIdx.z * per;
    const int64_t jend = min(W, jbeg + per);

    double acc[B][8];
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
        for (int v = 0; v < 8; ++v) acc[r][v] = 0.0;

    // generation role: thread t handles column (t & 63) for points wave, wave + WV, ...
    const int gcol = col0 + lane;
    const double theta = (2.0 * 3.141592653589793 * (double)gcol) / (double)d.n1;
    double sth, cth;
    sincos(theta, &sth, &cth);

    for (int64_t j0 = jbeg; j0 < jend; j0 += kPolarChunk) {
        const int nk = (int)min((int64_t)kPolarChunk, jend - j0);
        __syncthreads();
        for (int jj = wave; jj < kPolarChunk; jj += WV) {
            const bool ok = jj < nk;
            const double Y = ok ? pts[j0 + jj].Y : 0.0;
            const double Z = ok ? pts[j0 + jj].Z : 0.0;
            const double u = Y * sth + Z * cth;
            const double2 step = twiddle(d.step0 * u);
            double2 sb = cart::cmul(step, step);  // step^8: from one wave's rows to the next
            sb = cart::cmul(sb, sb);
            sb = cart::cmul(sb, sb);
            // start of the block: q(row0) = row0 dq, so exp(-i q(row0) u) = step^row0
            double2 st = cpow_int(sb, row0 / B);
            s_step[jj][lane] = step;
            s_k[jj][lane] = step.x + step.x;
#pragma unroll
            for (int w = 0; w < WV; ++w) {
                s_start[jj][w][lane] = st;
                st = cart::cmul(st, sb);
            }
        }
        if (t < kPolarChunk) {
            const bool ok = t < nk;
#pragma unroll
            for (int v = 0; v < 4; ++v) s_w[t][v] = ok ? pts[j0 + t].w[v] : 0.0;
        }
        __syncthreads();
        // operands of the next point are requested before the current point is
        // accumulated (as in the Cartesian loop)
        cart::Operands opa = polar_operands<WV>(s_start, s_step, s_k, s_w, 0, lane, wave);
        int jj = 0;
        for (; jj + 1 < nk; jj += 2) {
            const cart::Operands opb = polar_operands<WV>(s_start, s_step, s_k, s_w, jj + 1, lane, wave);
            __builtin_amdgcn_sched_barrier(0);
            polar_point<B>(opa, acc);
            __builtin_amdgcn_sched_barrier(0);
            opa = polar_operands<WV>(s_start, s_step, s_k, s_w, jj + 2, lane, wave);  // row kPolarChunk at most
            __builtin_amdgcn_sched_barrier(0);
            polar_point<B>(opb, acc);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (jj < nk) polar_point<B>(opa, acc);
    }
    const int64_t P = (int64_t)d.n0 * d.n1;
    double *dst = out + (int64_t)blockIdx.z * P * 8;
#pragma unroll
    for (int r = 0; r < B; ++r) {
        const int row = row0 + wave * B + r;
        if (row < d.n0 && gcol < d.n1) {
            double *o = dst + ((int64_t)row * d.n1 + gcol) * 8;
#pragma unroll
            for (int v = 0; v < 8; ++v) o[v] = acc[r][v];
        }
    }
}

// Waves per workgroup of the polar kernel: 8 (64 rows) unless the detector has
// at most 32 q rows.
static int polar_waves(const Detector &d) { return d.n0 > 4 * kPolarB ? 8 : 4; }

DirectPlan plan_direct_polar(const Detector &d, int64_t W)
{
    DirectPlan p{};
    p.lanes = 64;
    const int rows = polar_waves(d) * kPolarB;
    p.col_blocks = (d.n1 + 63) / 64;
    p.row_blocks = (d.n0 + rows - 1) / rows;
    int64_t blocks = (int64_t)p.col_blocks * p.row_blocks;
    int64_t want = (target_workgroups() * 4 / polar_waves(d) + blocks - 1) / blocks;
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
    if (polar_waves(d) == 8)
        hipLaunchKernelGGL(direct_polar_kernel<8>, grid, dim3(512), 0, s, pts, W, p.per, d, partial);
    else
        hipLaunchKernelGGL(direct_polar_kernel<4>, grid, dim3(256), 0, s, pts, W, p.per, d, partial);
    NUMAG_HIP_CHECK(hipGetLastError());
    return NUMAG_OK;
}

__global__ void fill_kernel(double *__restrict__ out, int64_t n, double value)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = value;
}

int launch_fill(double *out, int64_t n, double value, hipStream_t s)
{
    if (n <= 0) return NUMAG_OK;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n, value);
    NUMAG_HIP_CHECK(hipGetLastError());
    return NUMAG_OK;
}

// ---------------------------------------------------------------------------
// fixed-order FP64 combine of split partials.
// ---------------------------------------------------------------------------
__global__ void combine_kernel(const double *__restrict__ part, int nsplit, int64_t n,
                               double *__restrict__ out, int accumulate)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = accumulate ? out[i] : 0.0;
    for (int k = 0; k < nsplit; ++k) s += part[(int64_t)k * n + i];
    out[i] = s;
}

int launch_combine(const double *part, int nsplit, int64_t P, double *out, int accumulate,
                   hipStream_t s)
{
    int64_t n = P * 8;
    if (n <= 0) return NUMAG_OK;
    int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(combine_kernel, dim3((unsigned)blocks), dim3(256), 0, s, part, nsplit, n, out,
                       accumulate);
    NUMAG_HIP_CHECK(hipGetLastError());
    return NUMAG_OK;
}

}  // namespace numag
