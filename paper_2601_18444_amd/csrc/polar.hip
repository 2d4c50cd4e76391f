// Direct Fourier sums on the paper's polar (q, theta) detector (Sec. 3.2), on the
// building block of polar_sum.h.
#include "polar_sum.h"

namespace numag {

int polar_shape_rows(int shape)
{
    const polar::ShapeDesc &s = polar::kShapes[shape];
    return polar::kB * s.waves * (64 / s.cols);
}
int polar_shape_cols(int shape) { return polar::kShapes[shape].cols; }
int polar_shape_waves(int shape) { return polar::kShapes[shape].waves; }

struct PolarRecLoader {
    const PointRec *__restrict__ pts;
    __device__ __forceinline__ cart::PointPart load(int64_t j, int slot) const
    {
        const PointRec &r = pts[j];
        return cart::PointPart{r.Y, r.Z, r.w[slot]};
    }
};

// grid.z = rotation r of a group x split sp (nsp splits per rotation); the points of
// rotation r are pts[r wrot, (r + 1) wrot).  One rotation: wrot = W, nsp = grid.z.
template <int WV, int CW, int CHK, int NB, int CH>
__global__ __launch_bounds__(64 * WV, 8 / WV) void direct_polar_kernel(const PointRec *__restrict__ pts,
                                                                      int64_t wrot, int64_t per, int nsp, Detector d,
                                                                      double *__restrict__ out)
{
    using S = polar::Shape<WV, CW, CHK, NB>;
    __shared__ polar::Smem<WV, CW, CHK, NB> sm;
    const int col0 = blockIdx.x * CW;
    const int64_t rbase = (int64_t)(blockIdx.z / nsp) * wrot;
    const int64_t jbeg = rbase + (int64_t)(blockIdx.z % nsp) * per;
    const int64_t jend = min(rbase + wrot, jbeg + per);
    double acc[polar::kB][2 * CH];
#pragma unroll
    for (int r = 0; r < polar::kB; ++r)
#pragma unroll
        for (int v = 0; v < 2 * CH; ++v) acc[r][v] = 0.0;
    polar::accumulate<WV, CW, CHK, NB, CH>(PolarRecLoader{pts}, jbeg, jend, d, col0, (int)blockIdx.y, sm, acc);
    const int64_t P = (int64_t)d.n0 * d.n1;
    double *dst = out + (int64_t)blockIdx.z * P * 8;
    const int gcol = col0 + polar::lane_col<WV, CW>();
    const int row0 = (int)blockIdx.y * S::ROWS + polar::lane_group<WV, CW>() * polar::kB;
#pragma unroll
    for (int r = 0; r < polar::kB; ++r) {
        const int row = row0 + r;
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
        const double cost = cpad * rb * (10.3 * rows + 150.0 + 2.0 * rows / polar::kB);
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
    const polar::ShapeDesc &sd = polar::kShapes[p.shape];
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
    const polar::ShapeDesc &sd = polar::kShapes[p.shape];
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

}  // namespace numag
