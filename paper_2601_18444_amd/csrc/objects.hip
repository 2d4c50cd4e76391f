// Objects and orientations on gfx950 (Sec. 3.3 summation relation and dilute
// approximation; Sec. 3.1 sample rotation, extended to many orientations).
//
// Dilute and split modes need each object's amplitude F_k complete before its
// outer product F_k F_k^H is formed, so sums are not split over point ranges
// here.  A work item is (object slot, rotation group, pixel block): the
// workgroup sums every point of its objects for every rotation of its group
// with the Cartesian building block (FP64), then adds F F^H (and, in split
// mode, exp(-i q.R r^k) F for the coherent total) into a slot of FP64
// accumulators that no other item touches.  Items are sorted by cost and
// handed out by a persistent kernel through an atomic counter, so particles of
// very uneven size balance across the chip; slot contents are summed in a
// fixed order at the end, so results are reproducible bit for bit.
//
// Rotations are applied on the fly (X = R x, w' = (n, R m)) while a chunk's
// twiddles are generated, so the point data is read once per chunk and never
// rewritten per orientation.
#include <algorithm>
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
    const int4 *items;       // (kslot, h, block, -)
    const int2 *kslot_range; // object range of a slot
    const int2 *rot_range;   // rotation range of a group
    int n_items, n_kslots, col_blocks;
    int *counter;
    double *spec;            // [H][n_kslots][P][16]
    double *amp;             // [n_kslots][P][8] or null (split mode)
};

template <int A, int B>
__global__ __launch_bounds__(cart::kThreads, 2) void objects_kernel(ObjArgs a, Detector d)
{
    __shared__ cart::Smem<A> sm;
    __shared__ int s_item;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t P = (int64_t)d.n0 * d.n1;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= a.n_items) break;
        const int4 item = a.items[it];
        const int ks = item.x, h = item.y, blk = item.z;
        const int col0 = (blk % a.col_blocks) * 64 * B;
        const int row0 = (blk / a.col_blocks) * cart::kWaves * A;
        const int2 kr = a.kslot_range[ks];
        const int2 rr = a.rot_range[h];
        double *G = a.spec + ((int64_t)h * a.n_kslots + ks) * P * 16;
        for (int r = rr.x; r < rr.y; ++r) {
            const double *R = a.rot + 9 * (int64_t)r;
            for (int k = kr.x; k < kr.y; ++k) {
                double acc[A][B][8];
                cart::zero<A, B>(acc);
                cart::accumulate<A, B>(RawLoader{a.pos, a.nuc, a.mag, R}, a.off[k], a.off[k + 1], d, col0, row0,
                                       sm, acc);
                // lab position of the object (split mode)
                double XY = 0.0, XZ = 0.0;
                if (a.amp != nullptr && a.obj_pos != nullptr) {
                    const double *o = a.obj_pos + 3 * k;
                    XY = R[3] * o[0] + R[4] * o[1] + R[5] * o[2];
                    XZ = R[6] * o[0] + R[7] * o[1] + R[8] * o[2];
                }
#pragma unroll
                for (int rr2 = 0; rr2 < A; ++rr2) {
                    const int row = row0 + wave * A + rr2;
#pragma unroll
                    for (int c = 0; c < B; ++c) {
                        const int col = col0 + lane * B + c;
                        if (row >= d.n0 || col >= d.n1) continue;
                        const int64_t p = (int64_t)row * d.n1 + col;
                        const double *F = acc[rr2][c];
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
                            const double qy = cart::axis_value(d.origin0, row, d.step0);
                            const double qz = cart::axis_value(d.origin1, col, d.step1);
                            const double2 ph = cart::twiddle(qy * XY + qz * XZ);
                            double *o = a.amp + ((int64_t)ks * P + p) * 8;
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

// spec_out[s][p][v] = scale * sum over (h, kslot) mapped to s
__global__ void spec_reduce_kernel(const double *__restrict__ slots, int H, int n_kslots, int per_object,
                                   int64_t P, double scale, double *__restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n_out = (per_object ? n_kslots : 1) * P * 16;
    if (idx >= n_out) return;
    const int64_t pv = idx % (P * 16);
    double s = 0.0;
    if (per_object) {
        const int ks = (int)(idx / (P * 16));
        for (int h = 0; h < H; ++h) s += slots[((int64_t)h * n_kslots + ks) * P * 16 + pv];
    } else {
        for (int h = 0; h < H; ++h)
            for (int ks = 0; ks < n_kslots; ++ks) s += slots[((int64_t)h * n_kslots + ks) * P * 16 + pv];
    }
    out[idx] = scale * s;
}

__global__ void amp_reduce_kernel(const double *__restrict__ slots, int n_kslots, int64_t P,
                                  double *__restrict__ out)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= P * 8) return;
    double s = 0.0;
    for (int ks = 0; ks < n_kslots; ++ks) s += slots[(int64_t)ks * P * 8 + idx];
    out[idx] = s;
}

int device_cus()
{
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

// Host-side record of the tables last uploaded into a workspace, so that a
// repeated call (e.g. one recorded into a HIP graph) enqueues no host copy.
struct Upload {
    std::vector<char> bytes;
};
std::mutex g_upload_mu;
std::unordered_map<const void *, Upload> g_uploads;

}  // namespace

void forget_workspace(const void *ws)
{
    std::lock_guard<std::mutex> lk(g_upload_mu);
    g_uploads.erase(ws);
}

ObjectsPlan plan_objects(const Detector &d, const int64_t *h_off, int64_t K, int64_t n_rot, int mode,
                         int spec_per_object)
{
    ObjectsPlan p{};
    cart::choose_shape(d.n1, p.A, p.B);
    p.col_blocks = (d.n1 + 64 * p.B - 1) / (64 * p.B);
    p.row_blocks = (d.n0 + cart::kWaves * p.A - 1) / (cart::kWaves * p.A);
    const int64_t nblocks = (int64_t)p.col_blocks * p.row_blocks;
    int64_t H = (kTarget + K * nblocks - 1) / (K * nblocks);
    H = std::max<int64_t>(1, std::min<int64_t>(H, n_rot));
    if (mode == NUMAG_MODE_SPLIT) H = 1;
    p.H = (int)H;
    if (spec_per_object) {
        p.n_kslots = (int)K;
    } else {
        int64_t G = (kTarget + H * nblocks - 1) / (H * nblocks);
        p.n_kslots = (int)std::max<int64_t>(1, std::min<int64_t>(G, K));
    }
    p.n_items = (int64_t)p.n_kslots * p.H * nblocks;
    (void)h_off;
    return p;
}

size_t objects_workspace_bytes(const ObjectsPlan &p, const Detector &d, int64_t K, int64_t n_rot, int mode)
{
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t P = (size_t)d.n0 * d.n1;
    size_t b = 0;
    b += al((size_t)(K + 1) * sizeof(int64_t));
    b += al((size_t)n_rot * 9 * sizeof(double));
    b += al((size_t)p.n_items * sizeof(int4));
    b += al((size_t)p.n_kslots * sizeof(int2));
    b += al((size_t)p.H * sizeof(int2));
    b += al(sizeof(int) * 64);
    b += al((size_t)p.H * p.n_kslots * P * 16 * sizeof(double));
    if (mode == NUMAG_MODE_SPLIT) b += al((size_t)p.n_kslots * P * 8 * sizeof(double));
    return b;
}

int launch_objects(const numag_sample &s, const double *h_rot, int64_t n_rot, const Detector &d, int mode,
                   int spec_per_object, double *spec_out, double *amp_out, void *ws, size_t ws_bytes,
                   hipStream_t st)
{
    const int64_t K = s.n_objects;
    const int64_t W = s.n_points;
    std::vector<int64_t> off(K + 1);
    if (K == 1 || s.obj_offsets == nullptr) {
        off[0] = 0;
        off[1] = W;
    } else {
        std::memcpy(off.data(), s.obj_offsets, sizeof(int64_t) * (K + 1));
    }
    const ObjectsPlan p = plan_objects(d, off.data(), K, n_rot, mode, spec_per_object);
    const int64_t nblocks = (int64_t)p.col_blocks * p.row_blocks;
    const int64_t P = (int64_t)d.n0 * d.n1;

    // object ranges of the slots: single objects, or contiguous groups of
    // roughly equal point counts
    std::vector<int2> ksr(p.n_kslots);
    if (spec_per_object || p.n_kslots == K) {
        for (int64_t k = 0; k < p.n_kslots; ++k) ksr[k] = make_int2((int)k, (int)k + 1);
    } else {
        int64_t k = 0;
        for (int g = 0; g < p.n_kslots; ++g) {
            const int64_t target = (W * (g + 1)) / p.n_kslots;
            const int64_t k0 = k;
            while (k < K && (off[k + 1] <= target || k == k0)) ++k;
            if (g == p.n_kslots - 1) k = K;
            ksr[g] = make_int2((int)k0, (int)k);
        }
    }
    std::vector<int2> rr(p.H);
    for (int h = 0; h < p.H; ++h) rr[h] = make_int2((int)(n_rot * h / p.H), (int)(n_rot * (h + 1) / p.H));
    std::vector<int4> items;
    std::vector<int64_t> cost;
    items.reserve(p.n_items);
    for (int ks = 0; ks < p.n_kslots; ++ks)
        for (int h = 0; h < p.H; ++h)
            for (int64_t b = 0; b < nblocks; ++b) items.push_back(make_int4(ks, h, (int)b, 0));
    std::vector<int64_t> idx(items.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int64_t)i;
    auto item_cost = [&](const int4 &it) {
        return (off[ksr[it.x].y] - off[ksr[it.x].x] + 1) * (int64_t)(rr[it.y].y - rr[it.y].x);
    };
    std::stable_sort(idx.begin(), idx.end(),
                     [&](int64_t a, int64_t b) { return item_cost(items[a]) > item_cost(items[b]); });
    std::vector<int4> sorted(items.size());
    for (size_t i = 0; i < idx.size(); ++i) sorted[i] = items[idx[i]];

    // workspace layout
    char *base = (char *)ws;
    size_t used = 0;
    auto take = [&](size_t bytes) {
        char *r = base + used;
        used += (bytes + 255) & ~(size_t)255;
        return r;
    };
    char *tables = base;
    int64_t *d_off = (int64_t *)take(sizeof(int64_t) * (K + 1));
    double *d_rot = (double *)take(sizeof(double) * 9 * n_rot);
    int4 *d_items = (int4 *)take(sizeof(int4) * sorted.size());
    int2 *d_ksr = (int2 *)take(sizeof(int2) * ksr.size());
    int2 *d_rr = (int2 *)take(sizeof(int2) * rr.size());
    const size_t table_bytes = used;
    int *d_counter = (int *)take(sizeof(int) * 64);
    double *d_spec = (double *)take(sizeof(double) * 16 * (size_t)p.H * p.n_kslots * P);
    double *d_amp = mode == NUMAG_MODE_SPLIT ? (double *)take(sizeof(double) * 8 * (size_t)p.n_kslots * P) : nullptr;
    if (used > ws_bytes) {
        set_error("numag_amplitudes: workspace too small for the object path");
        return NUMAG_E_WORKSPACE;
    }

    // host image of the tables
    std::vector<char> img(table_bytes, 0);
    auto put = [&](const void *dst, const void *src, size_t n) {
        std::memcpy(img.data() + ((const char *)dst - tables), src, n);
    };
    put(d_off, off.data(), sizeof(int64_t) * (K + 1));
    if (h_rot != nullptr) {
        put(d_rot, h_rot, sizeof(double) * 9 * n_rot);
    } else {
        const double I3[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        put(d_rot, I3, sizeof(I3));
    }
    put(d_items, sorted.data(), sizeof(int4) * sorted.size());
    put(d_ksr, ksr.data(), sizeof(int2) * ksr.size());
    put(d_rr, rr.data(), sizeof(int2) * rr.size());
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
    int rc = launch_fill(d_spec, 16 * (int64_t)p.H * p.n_kslots * P, 0.0, st);
    if (rc != NUMAG_OK) return rc;
    if (d_amp != nullptr && (rc = launch_fill(d_amp, 8 * (int64_t)p.n_kslots * P, 0.0, st)) != NUMAG_OK) return rc;
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
    args.kslot_range = d_ksr;
    args.rot_range = d_rr;
    args.n_items = (int)p.n_items;
    args.n_kslots = p.n_kslots;
    args.col_blocks = p.col_blocks;
    args.counter = d_counter;
    args.spec = d_spec;
    args.amp = d_amp;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(p.n_items, 2LL * device_cus()));
    switch (p.B) {
        case 1: hipLaunchKernelGGL((objects_kernel<8, 1>), dim3((unsigned)grid), dim3(cart::kThreads), 0, st, args, d); break;
        case 2: hipLaunchKernelGGL((objects_kernel<4, 2>), dim3((unsigned)grid), dim3(cart::kThreads), 0, st, args, d); break;
        case 4: hipLaunchKernelGGL((objects_kernel<2, 4>), dim3((unsigned)grid), dim3(cart::kThreads), 0, st, args, d); break;
        default: hipLaunchKernelGGL((objects_kernel<1, 8>), dim3((unsigned)grid), dim3(cart::kThreads), 0, st, args, d); break;
    }
    NUMAG_HIP_CHECK(hipGetLastError());

    const int64_t n_spec = (spec_per_object ? p.n_kslots : 1) * P * 16;
    hipLaunchKernelGGL(spec_reduce_kernel, dim3((unsigned)((n_spec + 255) / 256)), dim3(256), 0, st, d_spec, p.H,
                       p.n_kslots, spec_per_object, P, 1.0 / (double)n_rot, spec_out);
    NUMAG_HIP_CHECK(hipGetLastError());
    if (d_amp != nullptr) {
        hipLaunchKernelGGL(amp_reduce_kernel, dim3((unsigned)((P * 8 + 255) / 256)), dim3(256), 0, st, d_amp,
                           p.n_kslots, P, amp_out);
        NUMAG_HIP_CHECK(hipGetLastError());
    }
    return NUMAG_OK;
}

}  // namespace numag
