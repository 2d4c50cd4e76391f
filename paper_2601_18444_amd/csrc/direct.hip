// Direct Fourier sums on gfx950, Cartesian detector: the general (any point
// cloud, any rotation) path, plus the point preparation and the split combine
// shared with the polar path (polar.hip).
//
// Sums (Sec. 3.3, DSFT):  S_c(q_p) = sum_j w_{j,c} exp(-i q_p . X_j),  q = (0, q_y, q_z).
//
// The phase separates in the lab frame, exp(-i (q_y Y + q_z Z)) =
// exp(-i q_y Y) exp(-i q_z Z); the tile layout, the twiddle generation and the
// two-term column recurrence are described in cartesian_sum.h.  There is no
// transcendental per term, and everything is accumulated in FP64 (FP32 phasors
// lose the 1e-5 gate at 10^-6 of the maximum on 2.6e5-point samples, however the
// sums are folded).
//
// Work is split over point ranges (split-K); a fixed-order FP64 combine sums
// the partial results, so results are bitwise reproducible.
#include <algorithm>

#include "cartesian_sum.h"

namespace numag {


Detector make_detector(const numag_qgrid &g)
{
    Detector d{};
    d.kind = g.kind;
    d.n0 = g.n0;
    d.n1 = g.n1;
    d.n_theta = g.n1;
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
// Lab-frame record of point j at sample-frame position x: X = R x (only Y, Z enter
// the phase), weights (n, R m).
__device__ __forceinline__ PointRec point_record(const double (&x)[3], const Rot &R, const double *__restrict__ nuc,
                                                 const double *__restrict__ mag, int64_t j)
{
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
    return r;
}

// Objects whose offsets r^k one preparation launch adds: the points
// [start[0], start[n]) belong to objects k0 .. k0 + n - 1, object k0 + i holding
// [start[i], start[i + 1]).  Passed by value, so no host-to-device copy is needed.
constexpr int kObjGroup = 64;
struct ObjGroup {
    int n;
    int64_t k0;
    int64_t start[kObjGroup + 1];
};

// Writes out[j - out_base] for the points j in [g.start[0], g.start[g.n]);
// obj_pos == nullptr: no object offsets.
__global__ void prepare_points_kernel(const double *__restrict__ pos, const double *__restrict__ nuc,
                                      const double *__restrict__ mag, int reg, numag_regular rg, ObjGroup g,
                                      const double *__restrict__ obj_pos, Rot R, int64_t out_base,
                                      PointRec *__restrict__ out)
{
    const int64_t j = g.start[0] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.start[g.n]) return;
    double x[3];
    if (reg) {
        int64_t nyz = (int64_t)rg.n[1] * rg.n[2];
        int64_t ix = j / nyz, rem = j % nyz;
        int64_t iy = rem / rg.n[2], iz = rem % rg.n[2];
        x[0] = rg.origin[0] + (double)ix * rg.step[0];
        x[1] = rg.origin[1] + (double)iy * rg.step[1];
        x[2] = rg.origin[2] + (double)iz * rg.step[2];
    } else {
        x[0] = pos[3 * j + 0];
        x[1] = pos[3 * j + 1];
        x[2] = pos[3 * j + 2];
    }
    if (obj_pos != nullptr) {
        int lo = 0, hi = g.n - 1;  // largest i with start[i] <= j
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (g.start[mid] <= j) lo = mid; else hi = mid - 1;
        }
        const int64_t k = g.k0 + lo;
        x[0] += obj_pos[3 * k + 0];
        x[1] += obj_pos[3 * k + 1];
        x[2] += obj_pos[3 * k + 2];
    }
    out[j - out_base] = point_record(x, R, nuc, mag, j);
}

int launch_prepare_points(const double *pos, const double *nuc, const double *mag, int64_t j_lo, int64_t j_hi,
                          const numag_regular *regular, const int64_t *h_offsets, int64_t K,
                          const double *obj_pos, const Rot &R, PointRec *out, hipStream_t s)
{
    if (j_hi <= j_lo) return NUMAG_OK;
    numag_regular rg{};
    if (regular != nullptr) rg = *regular;
    const int tpb = 256;
    auto launch = [&](const ObjGroup &g) -> int {
        const int64_t n = g.start[g.n] - g.start[0];
        if (n <= 0) return NUMAG_OK;
        hipLaunchKernelGGL(prepare_points_kernel, dim3((unsigned)((n + tpb - 1) / tpb)), dim3(tpb), 0, s, pos, nuc,
                           mag, regular != nullptr ? 1 : 0, rg, g, obj_pos, R, j_lo, out);
        NUMAG_HIP_CHECK(hipGetLastError());
        return NUMAG_OK;
    };
    ObjGroup g{};
    if (obj_pos == nullptr || K <= 1 || h_offsets == nullptr) {
        g.n = 1;
        g.k0 = 0;
        g.start[0] = j_lo;
        g.start[1] = j_hi;
        return launch(g);
    }
    // first object holding a point >= j_lo: the last k with off[k] <= j_lo among non-empty objects
    int64_t k = std::upper_bound(h_offsets, h_offsets + K + 1, j_lo) - h_offsets - 1;
    while (k < K && h_offsets[k + 1] <= j_lo) ++k;
    while (k < K && h_offsets[k] < j_hi) {
        g.n = 0;
        g.k0 = k;
        while (g.n < kObjGroup && k < K && h_offsets[k] < j_hi) {
            g.start[g.n] = std::max(h_offsets[k], j_lo);
            ++g.n;
            ++k;
        }
        g.start[g.n] = std::min(h_offsets[k], j_hi);
        const int rc = launch(g);
        if (rc != NUMAG_OK) return rc;
    }
    return NUMAG_OK;
}

// ---------------------------------------------------------------------------
// Cartesian direct sum.
// ---------------------------------------------------------------------------
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

template <int LR, int CH>
__global__ __launch_bounds__(kThreads, 2) void direct_cartesian_kernel(
    const PointRec *__restrict__ pts, int64_t W, int64_t per, Detector d, double *__restrict__ out)
{
    using T = cart::Tile<LR>;
    __shared__ cart::Smem<LR> sm;
    const int col0 = blockIdx.x * T::COLS;
    const int row0 = blockIdx.y * T::ROWS;
    const int64_t jbeg = (int64_t)blockIdx.z * per;
    const int64_t jend = min(W, jbeg + per);
    double acc[cart::kB][2 * CH];
    cart::zero(acc);
    cart::accumulate<LR, CH>(PrepLoader{pts}, jbeg, jend, d, col0, row0, sm, acc);

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
            for (int v = 0; v < 8; ++v) o[v] = cart::channel_value<CH>(acc[c], v);
        }
    }
}

int target_workgroups()
{
    static const int cached = [] {  // thread-safe one-time initialisation
        const char *e = getenv("NUMAG_TARGET_WGS");
        const int v = e != nullptr ? atoi(e) : 0;
        return v > 0 ? v : 2048;
    }();
    return cached;
}

TuneShape default_tune_shape(int kernel, const Detector &d, int64_t W)
{
    (void)W;
    switch (kernel) {
        case kTuneDirect:
            if (d.kind == NUMAG_GRID_POLAR) {
                const int sh = default_polar_shape(d);
                // half the Cartesian path's wave count: a polar workgroup of 8 waves holds
                // its CU alone, and two rounds of them over the chip measured faster than
                // four (fewer partials too)
                return TuneShape{sh, target_workgroups() * 2 / polar_shape_waves(sh)};
            }
            return TuneShape{cart::choose_lanes(d.n1), target_workgroups()};
        case kTuneAdjoint:
            // twice the direct path's workgroups (measured about 2 % faster than the same
            // count: shorter row ranges balance better across the CUs)
            return TuneShape{0, 2 * target_workgroups()};
        default:  // the persistent object kernel: lanes per row (polar: workgroup shape), work items
            if (d.kind == NUMAG_GRID_POLAR) return TuneShape{default_polar_shape(d), 1024};
            return TuneShape{cart::choose_lanes(d.n1), 2048};
    }
}

TuneShape current_tune_shape(int kernel, const Detector &d, int64_t W)
{
    TuneShape s{};
    if (tuned_shape(kernel, d, W, &s) && valid_tune_shape(kernel, d, s)) {
        if (s.target == 0) s.target = default_tune_shape(kernel, d, W).target;
        return s;
    }
    return default_tune_shape(kernel, d, W);
}

DirectPlan plan_direct_cartesian(const Detector &d, int64_t W, int64_t max_splits)
{
    DirectPlan p{};
    p.channels = 4;
    const TuneShape ts = current_tune_shape(kTuneDirect, d, W);
    p.lanes = ts.shape;
    const int cols = p.lanes * cart::kB, rows = kThreads / p.lanes;
    p.col_blocks = (d.n1 + cols - 1) / cols;
    p.row_blocks = (d.n0 + rows - 1) / rows;
    int64_t blocks = (int64_t)p.col_blocks * p.row_blocks;
    int64_t want = (ts.target + blocks - 1) / blocks;
    // each split should own a few chunks
    int64_t max_split = (W + 4 * kChunk - 1) / (4 * kChunk);
    if (max_split < 1) max_split = 1;
    if (want > max_split) want = max_split;
    if (max_splits > 0 && want > max_splits) want = max_splits;
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
#define NUMAG_LAUNCH_CART(LR, CH) \
    hipLaunchKernelGGL((direct_cartesian_kernel<LR, CH>), grid, block, 0, s, pts, W, p.per, d, partial)
#define NUMAG_LAUNCH_CART_CH(LR)                      \
    switch (p.channels) {                             \
        case 1: NUMAG_LAUNCH_CART(LR, 1); break;      \
        case 3: NUMAG_LAUNCH_CART(LR, 3); break;      \
        default: NUMAG_LAUNCH_CART(LR, 4); break;     \
    }
    switch (p.lanes) {
        case 8: NUMAG_LAUNCH_CART_CH(8); break;
        case 16: NUMAG_LAUNCH_CART_CH(16); break;
        case 32: NUMAG_LAUNCH_CART_CH(32); break;
        default: NUMAG_LAUNCH_CART_CH(64); break;
    }
#undef NUMAG_LAUNCH_CART_CH
#undef NUMAG_LAUNCH_CART
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

// ---------------------------------------------------------------------------
// Hermitian completion: for real weights S(-q) = conj S(q).  Cartesian: rows
// [0, h) of the row-major output are computed, pixel p mirrors to P - 1 - p.
// Polar (even n_theta): columns [0, n_theta / 2) are computed into a
// [n0][n_theta / 2] block, column m mirrors to m + n_theta / 2.
// ---------------------------------------------------------------------------
__global__ void mirror_cartesian_kernel(double *__restrict__ amp, int64_t P, int64_t Ph)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Ph * 8) return;
    const int64_t p = i >> 3;
    const int v = (int)(i & 7);
    const int64_t q = P - 1 - p;
    if (q >= Ph) amp[q * 8 + v] = (v & 1) ? -amp[i] : amp[i];
}

int launch_mirror_cartesian(double *amp, int64_t P, int64_t Ph, hipStream_t s)
{
    if (Ph <= 0) return NUMAG_OK;
    hipLaunchKernelGGL(mirror_cartesian_kernel, dim3((unsigned)((Ph * 8 + 255) / 256)), dim3(256), 0, s, amp, P, Ph);
    NUMAG_HIP_CHECK(hipGetLastError());
    return NUMAG_OK;
}

// out[i][m] = sum of the splits of part[.][i][m], out[i][m + nh] = its conjugate
__global__ void combine_polar_half_kernel(const double *__restrict__ part, int nsplit, int n0, int nh,
                                          double *__restrict__ out, int accumulate)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t Ph = (int64_t)n0 * nh;
    if (idx >= Ph * 8) return;
    const int64_t p = idx >> 3;
    const int v = (int)(idx & 7);
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += part[(int64_t)k * Ph * 8 + idx];
    const int64_t i = p / nh, m = p % nh;
    const int64_t full = i * 2 * nh + m;
    const double sm = (v & 1) ? -s : s;
    out[full * 8 + v] = accumulate ? out[full * 8 + v] + s : s;
    out[(full + nh) * 8 + v] = accumulate ? out[(full + nh) * 8 + v] + sm : sm;
}

int launch_combine_polar_half(const double *part, int nsplit, int n0, int nh, double *out, hipStream_t s,
                              int accumulate)
{
    const int64_t n = (int64_t)n0 * nh * 8;
    if (n <= 0) return NUMAG_OK;
    hipLaunchKernelGGL(combine_polar_half_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part, nsplit,
                       n0, nh, out, accumulate);
    NUMAG_HIP_CHECK(hipGetLastError());
    return NUMAG_OK;
}

}  // namespace numag
