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
// rewritten per orientation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "cartesian_sum.h"

namespace numag {

namespace {

constexpr int kTarget = 2048;  // work items aimed for

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

__global__ void fill_i32_kernel(int *p, int n, int v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// out[s][p][v] = scale * sum of the slots of output s (slot_off CSR, ascending);
// slots hold P pixels, out rows are P_out >= P pixels apart (the first P filled)
__global__ void spec_reduce_kernel(const double *__restrict__ slots, const int *__restrict__ slot_off, int n_out,
                                   int64_t P, int64_t P_out, double scale, double *__restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_out * P * 16) return;
    const int s = (int)(idx / (P * 16));
    const int64_t pv = idx % (P * 16);
    double acc = 0.0;
    for (int sl = slot_off[s]; sl < slot_off[s + 1]; ++sl) acc += slots[(int64_t)sl * P * 16 + pv];
    out[(int64_t)s * P_out * 16 + pv] = scale * acc;
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

__global__ void amp_reduce_kernel(const double *__restrict__ slots, int n_slots, int64_t P,
                                  double *__restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P * 8) return;
    double s = 0.0;
    for (int sl = 0; sl < n_slots; ++sl) s += slots[(int64_t)sl * P * 8 + idx];
    out[idx] = s;
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

// Host-side record of the tables last uploaded into a workspace, so that a
// repeated call (e.g. one recorded into a HIP graph) enqueues no host copy.
struct Upload {
    std::vector<char> bytes;
};
std::mutex g_upload_mu;
std::unordered_map<const void *, Upload> g_uploads;

// The full host-side plan: object groups, slots and sorted items.
struct Tables {
    ObjectsPlan p;
    std::vector<int64_t> off;     // [K+1]
    std::vector<int4> slots;      // (object lo, hi, rotation lo, hi)
    std::vector<int> slot_off;    // outputs -> slots (CSR)
    std::vector<int2> items;      // (slot, block), by decreasing cost
};

Tables make_tables(const Detector &d, const int64_t *h_off, int64_t K, int64_t W, int64_t n_rot, int mode,
                   int spec_per_object)
{
    Tables T;
    ObjectsPlan &p = T.p;
    p.lanes = cart::choose_lanes(d.n1);
    const int cols = p.lanes * cart::kB, rows = cart::kThreads / p.lanes;
    p.col_blocks = (d.n1 + cols - 1) / cols;
    p.row_blocks = (d.n0 + rows - 1) / rows;
    const int64_t nblocks = (int64_t)p.col_blocks * p.row_blocks;
    T.off.resize(K + 1);
    if (K == 1 || h_off == nullptr) {
        T.off[0] = 0;
        T.off[1] = W;
    } else {
        std::memcpy(T.off.data(), h_off, sizeof(int64_t) * (K + 1));
    }
    const std::vector<int64_t> &off = T.off;
    // slot groups wanted (each spans all pixel blocks)
    const int64_t want = std::max<int64_t>(1, (kTarget + nblocks - 1) / nblocks);
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

void forget_workspace(const void *ws)
{
    std::lock_guard<std::mutex> lk(g_upload_mu);
    g_uploads.erase(ws);
}

size_t objects_workspace_bytes(const Detector &d, const int64_t *h_off, int64_t K, int64_t W, int64_t n_rot,
                               int mode, int spec_per_object)
{
    const Tables T = make_tables(d, h_off, K, W, n_rot, mode, spec_per_object);
    const size_t P = (size_t)d.n0 * d.n1;
    size_t b = 0;
    b += al((size_t)(K + 1) * sizeof(int64_t));
    b += al((size_t)n_rot * 9 * sizeof(double));
    b += al(T.items.size() * sizeof(int2));
    b += al(T.slots.size() * sizeof(int4));
    b += al(T.slot_off.size() * sizeof(int));
    b += al(sizeof(int) * 64);
    b += al((size_t)T.p.n_slots * P * 16 * sizeof(double));
    if (mode == NUMAG_MODE_SPLIT) b += al((size_t)T.p.n_slots * P * 8 * sizeof(double));
    return b;
}

Detector objects_detector(const Detector &d, bool hermitian)
{
    Detector dk = d;
    if (hermitian) dk.n0 = (d.n0 + 1) / 2;  // rows [0, h): the first h n1 pixels of the outputs
    return dk;
}

int launch_objects(const numag_sample &s, const double *h_rot, int64_t n_rot, const Detector &d_full, int mode,
                   int spec_per_object, double *spec_out, double *amp_out, void *ws, size_t ws_bytes,
                   hipStream_t st, bool hermitian)
{
    const int64_t K = s.n_objects;
    const Detector d = objects_detector(d_full, hermitian);  // the rows that are summed
    const int64_t P = (int64_t)d.n0 * d.n1;
    const int64_t P_full = (int64_t)d_full.n0 * d_full.n1;
    const Tables T = make_tables(d, s.obj_offsets, K, s.n_points, n_rot, mode, spec_per_object);
    const ObjectsPlan &p = T.p;

    // workspace layout
    char *base = (char *)ws;
    size_t used = 0;
    auto take = [&](size_t bytes) {
        char *r = base + used;
        used += al(bytes);
        return r;
    };
    char *tables = base;
    int64_t *d_off = (int64_t *)take(sizeof(int64_t) * (K + 1));
    double *d_rot = (double *)take(sizeof(double) * 9 * n_rot);
    int2 *d_items = (int2 *)take(sizeof(int2) * T.items.size());
    int4 *d_slots = (int4 *)take(sizeof(int4) * T.slots.size());
    int *d_slot_off = (int *)take(sizeof(int) * T.slot_off.size());
    const size_t table_bytes = used;
    int *d_counter = (int *)take(sizeof(int) * 64);
    double *d_spec = (double *)take(sizeof(double) * 16 * (size_t)p.n_slots * P);
    double *d_amp = mode == NUMAG_MODE_SPLIT ? (double *)take(sizeof(double) * 8 * (size_t)p.n_slots * P) : nullptr;
    if (used > ws_bytes) {
        set_error("numag_amplitudes: workspace too small for the object path");
        return NUMAG_E_WORKSPACE;
    }

    // host image of the tables
    std::vector<char> img(table_bytes, 0);
    auto put = [&](const void *dst, const void *src, size_t n) {
        std::memcpy(img.data() + ((const char *)dst - tables), src, n);
    };
    put(d_off, T.off.data(), sizeof(int64_t) * (K + 1));
    if (h_rot != nullptr) {
        put(d_rot, h_rot, sizeof(double) * 9 * n_rot);
    } else {
        const double I3[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        put(d_rot, I3, sizeof(I3));
    }
    put(d_items, T.items.data(), sizeof(int2) * T.items.size());
    put(d_slots, T.slots.data(), sizeof(int4) * T.slots.size());
    put(d_slot_off, T.slot_off.data(), sizeof(int) * T.slot_off.size());
    bool upload = true;
    {
        std::lock_guard<std::mutex> lk(g_upload_mu);
        auto itr = g_uploads.find(ws);
        if (itr != g_uploads.end() && itr->second.bytes == img) upload = false;
    }
    if (upload) {
        NUMAG_HIP_CHECK(hipMemcpyAsync(tables, img.data(), img.size(), hipMemcpyHostToDevice, st));
        NUMAG_HIP_CHECK(hipStreamSynchronize(st));  // the host image goes out of scope
        std::lock_guard<std::mutex> lk(g_upload_mu);
        g_uploads[ws].bytes = img;
    }

    // zero the accumulators and the counter (kernels, so the sequence can be captured)
    int rc = launch_fill(d_spec, 16 * (int64_t)p.n_slots * P, 0.0, st);
    if (rc != NUMAG_OK) return rc;
    if (d_amp != nullptr && (rc = launch_fill(d_amp, 8 * (int64_t)p.n_slots * P, 0.0, st)) != NUMAG_OK) return rc;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, st, d_counter, 64, 0);
    NUMAG_HIP_CHECK(hipGetLastError());

    ObjArgs args{};
    args.pos = s.pos;
    args.nuc = s.nuc;
    args.mag = s.mag;
    args.off = d_off;
    args.obj_pos = s.obj_pos;
    args.rot = d_rot;
    args.items = d_items;
    args.slots = d_slots;
    args.n_items = (int)p.n_items;
    args.col_blocks = p.col_blocks;
    args.counter = d_counter;
    args.spec = d_spec;
    args.amp = d_amp;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(p.n_items, 2LL * device_cus()));
    {
        TimedLaunch timed(NUMAG_KERNEL_OBJECTS, st);
        switch (p.lanes) {
            case 8: hipLaunchKernelGGL((objects_kernel<8>), dim3((unsigned)grid), dim3(cart::kThreads), 0, st, args, d); break;
            case 16: hipLaunchKernelGGL((objects_kernel<16>), dim3((unsigned)grid), dim3(cart::kThreads), 0, st, args, d); break;
            case 32: hipLaunchKernelGGL((objects_kernel<32>), dim3((unsigned)grid), dim3(cart::kThreads), 0, st, args, d); break;
            default: hipLaunchKernelGGL((objects_kernel<64>), dim3((unsigned)grid), dim3(cart::kThreads), 0, st, args, d); break;
        }
    }
    NUMAG_HIP_CHECK(hipGetLastError());

    const int64_t n_spec = (int64_t)p.n_out * P * 16;
    hipLaunchKernelGGL(spec_reduce_kernel, dim3((unsigned)((n_spec + 255) / 256)), dim3(256), 0, st, d_spec, d_slot_off,
                       p.n_out, P, P_full, 1.0 / (double)n_rot, spec_out);
    NUMAG_HIP_CHECK(hipGetLastError());
    if (d_amp != nullptr) {
        hipLaunchKernelGGL(amp_reduce_kernel, dim3((unsigned)((P * 8 + 255) / 256)), dim3(256), 0, st, d_amp,
                           p.n_slots, P, amp_out);
        NUMAG_HIP_CHECK(hipGetLastError());
    }
    if (hermitian) {
        hipLaunchKernelGGL(mirror_spec_kernel, dim3((unsigned)((n_spec + 255) / 256)), dim3(256), 0, st, spec_out,
                           p.n_out, P_full, P);
        NUMAG_HIP_CHECK(hipGetLastError());
        if (amp_out != nullptr && d_amp != nullptr) return launch_mirror_cartesian(amp_out, P_full, P, st);
    }
    return NUMAG_OK;
}

}  // namespace numag
