// Objects and orientations on gfx950 (Sec. 3.3 summation relation and dilute
// approximation; Sec. 3.1 sample rotation, extended to many orientations).
//
// Dilute and split modes need each object's amplitude F_k complete before its
// outer product F_k F_k^H is formed, so sums are not split over point ranges
// here.  The work is cut into accumulator slots: a slot is a set of objects
// (one object, or a contiguous group of roughly equal point count) and a range
// of rotations, sized so that every slot costs about the same; a large particle
// gets many rotation ranges, a small one a single range.  A work item is
// (slot, pixel block): the workgroup sums every point of the slot's objects for
// every rotation of its range with the Cartesian building block (FP64), then
// adds F F^H (and, in split mode, exp(-i q.R r^k) F for the coherent total)
// into the slot's FP64 accumulators, which no other item touches.  Items are
// sorted by cost and handed out by a persistent kernel through an atomic
// counter; slots are reduced in a fixed order, so results are reproducible
// bit for bit.
//
// Rotations are applied on the fly (X = R x, w' = (n, R m)) while a chunk's
// twiddles are generated, so the point data is read once per chunk and never
// rewritten per orientation.  On a polar detector the same work queue runs on the
// polar building block (polar_sum.h): a pixel block is one of its workgroup
// tiles (q rows x theta columns).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "cartesian_sum.h"
#include "polar_sum.h"

namespace numag {

namespace {

struct RawLoader {
    const double *pos, *nuc, *mag;
    const double *R;  // row-major 3x3, wave-uniform
    __device__ __forceinline__ cart::PointPart load(int64_t j, int slot) const
    {
        const double x0 = pos[3 * j], x1 = pos[3 * j + 1], x2 = pos[3 * j + 2];
        cart::PointPart p;
        p.Y = R[3] * x0 + R[4] * x1 + R[5] * x2;
        p.Z = R[6] * x0 + R[7] * x1 + R[8] * x2;
        p.w = 0.0;
        if (slot == 0) {
            p.w = nuc != nullptr ? nuc[j] : 0.0;
        } else if (slot < 4 && mag != nullptr) {
            const int a = slot - 1;
            p.w = R[3 * a] * mag[3 * j] + R[3 * a + 1] * mag[3 * j + 1] + R[3 * a + 2] * mag[3 * j + 2];
        }
        return p;
    }
};

struct ObjArgs {
    const unsigned long long *tag_ptr;  // the plan tag at the start of the workspace
    unsigned long long tag;             // the tag of the plan these tables belong to
    const double *pos, *nuc, *mag;
    const int64_t *off;      // [K+1]
    const double *obj_pos;   // [K][3] or null
    const double *rot;       // [n_rot][9]
    const int2 *items;       // (slot, pixel block), sorted by cost
    const int4 *slots;       // (object lo, object hi, rotation lo, rotation hi)
    int n_items, col_blocks;
    int *counter;
    double *spec;            // [n_slots][P][16]
    double *amp;             // [n_slots][P][8] or null (split mode)
};

template <int LR>
__global__ __launch_bounds__(cart::kThreads, 2) void objects_kernel(ObjArgs a, Detector d)
{
    using T = cart::Tile<LR>;
    __shared__ cart::Smem<LR> sm;
    __shared__ int s_item;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t P = (int64_t)d.n0 * d.n1;
    if (*a.tag_ptr != a.tag) return;  // the workspace does not hold this plan's tables
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= a.n_items) break;
        const int2 item = a.items[it];
        const int slot = item.x, blk = item.y;
        const int col0 = (blk % a.col_blocks) * T::COLS;
        const int row0 = (blk / a.col_blocks) * T::ROWS;
        const int row = T::row(row0, lane, wave);
        const int4 sr = a.slots[slot];
        double *G = a.spec + (int64_t)slot * P * 16;
        for (int r = sr.z; r < sr.w; ++r) {
            const double *R = a.rot + 9 * (int64_t)r;
            for (int k = sr.x; k < sr.y; ++k) {
                double acc[cart::kB][8];
                cart::zero(acc);
                cart::accumulate<LR>(RawLoader{a.pos, a.nuc, a.mag, R}, a.off[k], a.off[k + 1], d, col0, row0, sm,
                                     acc);
                // lab position of the object (split mode)
                double XY = 0.0, XZ = 0.0;
                if (a.amp != nullptr && a.obj_pos != nullptr) {
                    const double *o = a.obj_pos + 3 * k;
                    XY = R[3] * o[0] + R[4] * o[1] + R[5] * o[2];
                    XZ = R[6] * o[0] + R[7] * o[1] + R[8] * o[2];
                }
                {
#pragma unroll
                    for (int c = 0; c < cart::kB; ++c) {
                        const int col = T::col(col0, lane, c);
                        if (row >= d.n0 || col >= d.n1) continue;
                        const int64_t p = (int64_t)row * d.n1 + col;
                        const double *F = acc[c];
                        double *g = G + p * 16;
                        // G_ab += F_a conj(F_b): diagonal, then the upper triangle
                        g[0] += F[0] * F[0] + F[1] * F[1];
                        g[1] += F[2] * F[2] + F[3] * F[3];
                        g[2] += F[4] * F[4] + F[5] * F[5];
                        g[3] += F[6] * F[6] + F[7] * F[7];
                        const int pa[6] = {0, 0, 0, 1, 1, 2};
                        const int pb[6] = {1, 2, 3, 2, 3, 3};
#pragma unroll
                        for (int t = 0; t < 6; ++t) {
                            const double ar = F[2 * pa[t]], ai = F[2 * pa[t] + 1];
                            const double br = F[2 * pb[t]], bi = F[2 * pb[t] + 1];
                            g[4 + 2 * t] += ar * br + ai * bi;
                            g[5 + 2 * t] += ai * br - ar * bi;
                        }
                        if (a.amp != nullptr) {
                            const double qy = axis_value(d.origin0, row, d.step0);
                            const double qz = axis_value(d.origin1, col, d.step1);
                            const double2 ph = twiddle(qy * XY + qz * XZ);
                            double *o = a.amp + ((int64_t)slot * P + p) * 8;
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                o[2 * v] += ph.x * F[2 * v] - ph.y * F[2 * v + 1];
                                o[2 * v + 1] += ph.x * F[2 * v + 1] + ph.y * F[2 * v];
                            }
                        }
                    }
                }
            }
        }
    }
}

// The same work queue on a polar detector: a pixel block is a polar workgroup
// tile (col_blocks theta-column blocks of CW columns x row blocks of ROWS q rows);
// the lane's pixels are its 8 q rows of one theta column.
template <int WV, int CW, int CHK, int NB>
__global__ __launch_bounds__(64 * WV, 8 / WV) void objects_polar_kernel(ObjArgs a, Detector d)
{
    using S = polar::Shape<WV, CW, CHK, NB>;
    __shared__ polar::Smem<WV, CW, CHK, NB> sm;
    __shared__ int s_item;
    const int64_t P = (int64_t)d.n0 * d.n1;
    if (*a.tag_ptr != a.tag) return;  // the workspace does not hold this plan's tables
    const int lc = polar::lane_col<WV, CW>(), lg = polar::lane_group<WV, CW>();
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= a.n_items) break;
        const int2 item = a.items[it];
        const int slot = item.x, blk = item.y;
        const int col0 = (blk % a.col_blocks) * CW;
        const int rb = blk / a.col_blocks;
        const int col = col0 + lc;
        const int row0 = rb * S::ROWS + lg * polar::kB;
        const int4 sr = a.slots[slot];
        double *G = a.spec + (int64_t)slot * P * 16;
        for (int r = sr.z; r < sr.w; ++r) {
            const double *R = a.rot + 9 * (int64_t)r;
            for (int k = sr.x; k < sr.y; ++k) {
                double acc[polar::kB][8];
#pragma unroll
                for (int q = 0; q < polar::kB; ++q)
#pragma unroll
                    for (int v = 0; v < 8; ++v) acc[q][v] = 0.0;
                polar::accumulate<WV, CW, CHK, NB, 4>(RawLoader{a.pos, a.nuc, a.mag, R}, a.off[k], a.off[k + 1], d,
                                                      col0, rb, sm, acc);
                if (col >= d.n1) continue;
                // lab position of the object projected on the column direction (split mode)
                double uk = 0.0;
                if (a.amp != nullptr && a.obj_pos != nullptr) {
                    const double *o = a.obj_pos + 3 * k;
                    const double XY = R[3] * o[0] + R[4] * o[1] + R[5] * o[2];
                    const double XZ = R[6] * o[0] + R[7] * o[1] + R[8] * o[2];
                    const double2 tr = sm.trig[lc];  // valid until the next accumulate call
                    uk = XY * tr.x + XZ * tr.y;
                }
#pragma unroll
                for (int q = 0; q < polar::kB; ++q) {
                    const int row = row0 + q;
                    if (row >= d.n0) break;
                    const int64_t p = (int64_t)row * d.n1 + col;
                    const double *F = acc[q];
                    double *g = G + p * 16;
                    // G_ab += F_a conj(F_b): diagonal, then the upper triangle
                    g[0] += F[0] * F[0] + F[1] * F[1];
                    g[1] += F[2] * F[2] + F[3] * F[3];
                    g[2] += F[4] * F[4] + F[5] * F[5];
                    g[3] += F[6] * F[6] + F[7] * F[7];
                    const int pa[6] = {0, 0, 0, 1, 1, 2};
                    const int pb[6] = {1, 2, 3, 2, 3, 3};
#pragma unroll
                    for (int t = 0; t < 6; ++t) {
                        const double ar = F[2 * pa[t]], ai = F[2 * pa[t] + 1];
                        const double br = F[2 * pb[t]], bi = F[2 * pb[t] + 1];
                        g[4 + 2 * t] += ar * br + ai * bi;
                        g[5 + 2 * t] += ai * br - ar * bi;
                    }
                    if (a.amp != nullptr) {
                        const double2 ph = twiddle(axis_value(d.origin0, row, d.step0) * uk);
                        double *o = a.amp + ((int64_t)slot * P + p) * 8;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            o[2 * v] += ph.x * F[2 * v] - ph.y * F[2 * v + 1];
                            o[2 * v + 1] += ph.x * F[2 * v + 1] + ph.y * F[2 * v];
                        }
                    }
                }
            }
        }
    }
}

__global__ void fill_i32_kernel(int *p, int n, int v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Full-detector pixel of pixel p of the evaluated part: the same index (the
// first rows of a Cartesian detector), or, with nh > 0, column p % nh of row
// p / nh of a polar detector of 2 nh columns (the half theta < pi).
__device__ __forceinline__ int64_t full_pixel(int64_t p, int nh)
{
    return nh > 0 ? (p / nh) * 2 * nh + p % nh : p;
}

// out[s][p][v] = scale * sum of the slots of output s (slot_off CSR, ascending);
// slots hold P pixels, out rows are P_out >= P pixels apart.  nh > 0: the slots
// hold the half theta < pi of a polar detector, and pixel (i, m + nh) receives
// conj G of pixel (i, m) (real weights: G(-q) = conj G(q)).
// A workspace that does not hold the plan's tables (tag mismatch) gives NaN.
__global__ void spec_reduce_kernel(const unsigned long long *tag_ptr, unsigned long long tag,
                                   const double *__restrict__ slots, const int *__restrict__ slot_off, int n_out,
                                   int64_t P, int64_t P_out, int nh, double scale, double *__restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_out * P * 16) return;
    const int s = (int)(idx / (P * 16));
    const int64_t pv = idx % (P * 16);
    const int v = (int)(pv & 15);
    const int64_t pf = full_pixel(pv >> 4, nh);
    double *o = out + (int64_t)s * P_out * 16;
    double val;
    if (*tag_ptr != tag) {
        val = __builtin_nan("");
    } else {
        double acc = 0.0;
        for (int sl = slot_off[s]; sl < slot_off[s + 1]; ++sl) acc += slots[(int64_t)sl * P * 16 + pv];
        val = scale * acc;
    }
    o[pf * 16 + v] = val;
    if (nh > 0) o[(pf + nh) * 16 + v] = (v >= 5 && (v & 1)) ? -val : val;
}

// out[i] = NaN for i < n when the workspace tag is not the plan's.
__global__ void tag_guard_kernel(const unsigned long long *tag_ptr, unsigned long long tag, double *out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && *tag_ptr != tag) out[i] = __builtin_nan("");
}

// Hermitian completion of spectral matrices on a centro-symmetric Cartesian
// detector: pixel P - 1 - p sits at -q(p), and with real weights
// G(-q) = conj G(q): the real diagonal is copied, the imaginary parts of the six
// upper entries (odd v >= 5) change sign.  Pixels [0, Ph) are given.
__global__ void mirror_spec_kernel(double *__restrict__ out, int n_out, int64_t P, int64_t Ph)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_out * Ph * 16) return;
    const int s = (int)(idx / (Ph * 16));
    const int64_t pv = idx % (Ph * 16);
    const int64_t p = pv >> 4;
    const int v = (int)(pv & 15);
    const int64_t q = P - 1 - p;
    if (q < Ph) return;
    double *o = out + (int64_t)s * P * 16;
    o[q * 16 + v] = (v >= 5 && (v & 1)) ? -o[p * 16 + v] : o[p * 16 + v];
}

// Coherent total: out = sum of the amplitude slots in order (nh > 0: polar half,
// pixel (i, m + nh) receives conj A of pixel (i, m)).
__global__ void amp_reduce_kernel(const unsigned long long *tag_ptr, unsigned long long tag,
                                  const double *__restrict__ slots, int n_slots, int64_t P, int nh,
                                  double *__restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P * 8) return;
    const int v = (int)(idx & 7);
    const int64_t pf = full_pixel(idx >> 3, nh);
    double val;
    if (*tag_ptr != tag) {
        val = __builtin_nan("");
    } else {
        double s = 0.0;
        for (int sl = 0; sl < n_slots; ++sl) s += slots[(int64_t)sl * P * 8 + idx];
        val = s;
    }
    out[pf * 8 + v] = val;
    if (nh > 0) out[(pf + nh) * 8 + v] = (v & 1) ? -val : val;
}

int device_cus()
{
    static const int cus = [] {  // thread-safe one-time initialisation
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        return n;
    }();
    return cus;
}

// The full host-side plan: object groups, slots and sorted items.
struct Tables {
    ObjectsPlan p;
    std::vector<int4> slots;      // (object lo, hi, rotation lo, hi)
    std::vector<int> slot_off;    // outputs -> slots (CSR)
    std::vector<int2> items;      // (slot, block), by decreasing cost
};

Tables make_tables(const Detector &d, const std::vector<int64_t> &off, int64_t K, int64_t W, int64_t n_rot, int mode,
                   int spec_per_object)
{
    Tables T;
    ObjectsPlan &p = T.p;
    const TuneShape ts = current_tune_shape(kTuneObjects, d, W);
    p.lanes = ts.shape;  // Cartesian: lanes per row; polar: the workgroup shape
    const int cols = d.kind == NUMAG_GRID_POLAR ? polar_shape_cols(p.lanes) : p.lanes * cart::kB;
    const int rows = d.kind == NUMAG_GRID_POLAR ? polar_shape_rows(p.lanes) : cart::kThreads / p.lanes;
    p.col_blocks = (d.n1 + cols - 1) / cols;
    p.row_blocks = (d.n0 + rows - 1) / rows;
    const int64_t nblocks = (int64_t)p.col_blocks * p.row_blocks;
    // slot groups wanted (each spans all pixel blocks)
    const int64_t want = std::max<int64_t>(1, (ts.target + nblocks - 1) / std::max<int64_t>(nblocks, 1));
    // object groups: single objects, or contiguous groups of roughly equal point counts
    std::vector<int2> groups;
    if (spec_per_object) {
        for (int64_t k = 0; k < K; ++k) groups.push_back(make_int2((int)k, (int)k + 1));
    } else {
        const int64_t G = std::max<int64_t>(1, std::min<int64_t>(want, K));
        int64_t k = 0;
        for (int64_t g = 0; g < G && k < K; ++g) {
            const int64_t target = (W * (g + 1)) / G;
            const int64_t k0 = k;
            while (k < K && (off[k + 1] <= target || k == k0)) ++k;
            if (g == G - 1) k = K;
            groups.push_back(make_int2((int)k0, (int)k));
        }
    }
    // rotation ranges per group, proportional to the group's cost
    const double total = (double)std::max<int64_t>(W, 1) * (double)n_rot;
    const double per_slot = total / (double)std::max<int64_t>(want, (int64_t)groups.size());
    T.slot_off.push_back(0);
    for (const int2 &g : groups) {
        const double cost = (double)(off[g.y] - off[g.x] + 1) * (double)n_rot;
        int64_t H = (int64_t)std::ceil(cost / per_slot);
        H = std::max<int64_t>(1, std::min<int64_t>(H, n_rot));
        if (mode == NUMAG_MODE_SPLIT) H = 1;
        for (int64_t h = 0; h < H; ++h)
            T.slots.push_back(make_int4(g.x, g.y, (int)(n_rot * h / H), (int)(n_rot * (h + 1) / H)));
        if (spec_per_object) T.slot_off.push_back((int)T.slots.size());
    }
    if (!spec_per_object) T.slot_off.push_back((int)T.slots.size());
    p.n_slots = (int)T.slots.size();
    p.n_out = spec_per_object ? (int)K : 1;
    // items, most expensive first
    std::vector<std::pair<int64_t, int2>> it;
    it.reserve((size_t)p.n_slots * nblocks);
    for (int s = 0; s < p.n_slots; ++s) {
        const int4 sl = T.slots[s];
        const int64_t cost = (off[sl.y] - off[sl.x] + 1) * (int64_t)(sl.w - sl.z);
        for (int64_t b = 0; b < nblocks; ++b) it.push_back({cost, make_int2(s, (int)b)});
    }
    std::stable_sort(it.begin(), it.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
    for (auto &x : it) T.items.push_back(x.second);
    p.n_items = (int64_t)T.items.size();
    return T;
}

size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

// The persistent kernel's part of an object-mode plan: the work tables and where
// they and the accumulators sit in the workspace.
struct ObjPlanTables {
    Tables T;
    Detector dk;  // the part of the detector that is summed
    size_t o_off, o_items, o_slots, o_slot_off, o_counter, o_spec, o_amp;
};

int launch_tag_guard(const unsigned long long *tag_ptr, unsigned long long tag, double *out, int64_t n, hipStream_t st)
{
    if (n <= 0) return NUMAG_OK;
    hipLaunchKernelGGL(tag_guard_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, tag_ptr, tag, out, n);
    NUMAG_HIP_CHECK(hipGetLastError());
    return NUMAG_OK;
}

Detector objects_detector(const Detector &d, bool hermitian)
{
    Detector dk = d;
    if (hermitian) {
        if (d.kind == NUMAG_GRID_CARTESIAN) dk.n0 = (d.n0 + 1) / 2;  // rows [0, h): the first h n1 pixels
        else dk.n1 = d.n1 / 2;  // theta in [0, pi); n_theta stays the full count
    }
    return dk;
}

void build_objects_plan(ObjPlan &pl)
{
    auto c = std::make_shared<ObjPlanTables>();
    c->dk = objects_detector(pl.d, pl.path == NUMAG_PATH_DIRECT_HERMITIAN);
    c->T = make_tables(c->dk, pl.off, pl.K, pl.W, pl.n_rot, pl.mode, pl.spec_per_object);
    const Tables &T = c->T;
    const size_t P = (size_t)c->dk.n0 * c->dk.n1;
    size_t used = kPlanTagBytes;
    auto take = [&](size_t bytes) {
        const size_t r = used;
        used += al(bytes);
        return r;
    };
    c->o_off = take(sizeof(int64_t) * (pl.K + 1));
    pl.o_rot = take(sizeof(double) * 9 * pl.n_rot);
    c->o_items = take(sizeof(int2) * T.items.size());
    c->o_slots = take(sizeof(int4) * T.slots.size());
    c->o_slot_off = take(sizeof(int) * T.slot_off.size());
    const size_t image_bytes = used;
    c->o_counter = take(sizeof(int) * 64);
    c->o_spec = take(sizeof(double) * 16 * (size_t)T.p.n_slots * P);
    c->o_amp = pl.mode == NUMAG_MODE_SPLIT ? take(sizeof(double) * 8 * (size_t)T.p.n_slots * P) : 0;
    pl.ws_bytes = used;
    // host image of the tag and the tables (rotations are filled by the caller)
    pl.image.assign(image_bytes, 0);
    std::memcpy(pl.image.data(), &pl.tag, sizeof(pl.tag));
    std::memcpy(pl.image.data() + c->o_off, pl.off.data(), sizeof(int64_t) * (pl.K + 1));
    std::memcpy(pl.image.data() + c->o_items, T.items.data(), sizeof(int2) * T.items.size());
    std::memcpy(pl.image.data() + c->o_slots, T.slots.data(), sizeof(int4) * T.slots.size());
    std::memcpy(pl.image.data() + c->o_slot_off, T.slot_off.data(), sizeof(int) * T.slot_off.size());
    pl.tables = c;
}

int launch_objects_plan(const ObjPlan &pl, const numag_sample &s, double *spec_out, double *amp_out, void *ws,
                        hipStream_t st)
{
    const ObjPlanTables &c = *pl.tables;
    const ObjectsPlan &p = c.T.p;
    const Detector &d = c.dk;
    const bool hermitian = pl.path == NUMAG_PATH_DIRECT_HERMITIAN;
    const int64_t P = (int64_t)d.n0 * d.n1;
    const int64_t P_full = (int64_t)pl.d.n0 * pl.d.n1;
    char *base = (char *)ws;
    const unsigned long long *tag_ptr = (const unsigned long long *)base;
    const unsigned long long tag = pl.tag;
    int *d_counter = (int *)(base + c.o_counter);
    double *d_spec = (double *)(base + c.o_spec);
    double *d_amp = pl.mode == NUMAG_MODE_SPLIT ? (double *)(base + c.o_amp) : nullptr;

    // zero the accumulators and the counter (kernels, so the sequence can be captured)
    int rc = launch_fill(d_spec, 16 * (int64_t)p.n_slots * P, 0.0, st);
    if (rc != NUMAG_OK) return rc;
    if (d_amp != nullptr && (rc = launch_fill(d_amp, 8 * (int64_t)p.n_slots * P, 0.0, st)) != NUMAG_OK) return rc;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, st, d_counter, 64, 0);
    NUMAG_HIP_CHECK(hipGetLastError());

    ObjArgs args{};
    args.tag_ptr = tag_ptr;
    args.tag = tag;
    args.pos = s.pos;
    args.nuc = s.nuc;
    args.mag = s.mag;
    args.off = (const int64_t *)(base + c.o_off);
    args.obj_pos = s.obj_pos;
    args.rot = (const double *)(base + pl.o_rot);
    args.items = (const int2 *)(base + c.o_items);
    args.slots = (const int4 *)(base + c.o_slots);
    args.n_items = (int)p.n_items;
    args.col_blocks = p.col_blocks;
    args.counter = d_counter;
    args.spec = d_spec;
    args.amp = d_amp;
    const bool pol = d.kind == NUMAG_GRID_POLAR;
    // persistent grid: as many workgroups as fit the chip at once
    const int per_cu = pol ? (polar_shape_waves(p.lanes) == 4 ? 2 : 1) : 2;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(p.n_items, (int64_t)per_cu * device_cus()));
    {
        TimedLaunch timed(NUMAG_KERNEL_OBJECTS, st);
        const dim3 g((unsigned)grid);
        if (pol) {
            switch (p.lanes) {
                case 0: hipLaunchKernelGGL((objects_polar_kernel<8, 64, 8, 2>), g, dim3(512), 0, st, args, d); break;
                case 1: hipLaunchKernelGGL((objects_polar_kernel<4, 64, 8, 1>), g, dim3(256), 0, st, args, d); break;
                case 2: hipLaunchKernelGGL((objects_polar_kernel<8, 32, 8, 2>), g, dim3(512), 0, st, args, d); break;
                case 3: hipLaunchKernelGGL((objects_polar_kernel<8, 16, 16, 1>), g, dim3(512), 0, st, args, d); break;
                default: hipLaunchKernelGGL((objects_polar_kernel<8, 16, 8, 2>), g, dim3(512), 0, st, args, d); break;
            }
        } else {
            switch (p.lanes) {
                case 8: hipLaunchKernelGGL((objects_kernel<8>), g, dim3(cart::kThreads), 0, st, args, d); break;
                case 16: hipLaunchKernelGGL((objects_kernel<16>), g, dim3(cart::kThreads), 0, st, args, d); break;
                case 32: hipLaunchKernelGGL((objects_kernel<32>), g, dim3(cart::kThreads), 0, st, args, d); break;
                default: hipLaunchKernelGGL((objects_kernel<64>), g, dim3(cart::kThreads), 0, st, args, d); break;
            }
        }
    }
    NUMAG_HIP_CHECK(hipGetLastError());

    // the half of a polar detector is mirrored by the reductions, that of a
    // Cartesian one by the mirror kernels below
    const int nh = pol && hermitian ? d.n1 : 0;
    const int64_t n_spec = (int64_t)p.n_out * P * 16;
    hipLaunchKernelGGL(spec_reduce_kernel, dim3((unsigned)((n_spec + 255) / 256)), dim3(256), 0, st, tag_ptr, tag,
                       d_spec, (const int *)(base + c.o_slot_off), p.n_out, P, P_full, nh, 1.0 / (double)pl.n_rot,
                       spec_out);
    NUMAG_HIP_CHECK(hipGetLastError());
    if (d_amp != nullptr) {
        hipLaunchKernelGGL(amp_reduce_kernel, dim3((unsigned)((P * 8 + 255) / 256)), dim3(256), 0, st, tag_ptr, tag,
                           d_amp, p.n_slots, P, nh, amp_out);
        NUMAG_HIP_CHECK(hipGetLastError());
    }
    if (hermitian && !pol) {
        hipLaunchKernelGGL(mirror_spec_kernel, dim3((unsigned)((n_spec + 255) / 256)), dim3(256), 0, st, spec_out,
                           p.n_out, P_full, P);
        NUMAG_HIP_CHECK(hipGetLastError());
        if (amp_out != nullptr && d_amp != nullptr) return launch_mirror_cartesian(amp_out, P_full, P, st);
    }
    return NUMAG_OK;
}

}  // namespace numag
