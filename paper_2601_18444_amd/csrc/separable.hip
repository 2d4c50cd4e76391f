// Regular-grid separable path on the gfx950 matrix cores.
//
// For points on a regular grid (micromagnetic cells) with no sample rotation,
// the lab phase q.r = q_y y + q_z z does not involve x, so the DSFT of Sec. 3.3
// factors exactly:
//   S_c(y, z)   = sum_x w_c(x, y, z)                      (projection along the beam)
//   T_c(y, k)   = sum_z S_c(y, z) exp(-i q_z(k) z)         (real x complex contraction)
//   F_c(i, k)   = sum_y exp(-i q_y(i) y) T_c(y, k)         (complex x complex contraction)
// The two contractions are dense GEMMs and run on MFMA:
//   NUMAG_PATH_SEPARABLE_F64:    FP64 operands and accumulation on
//                                v_mfma_f64_16x16x4f64 (_HERMITIAN: the second
//                                contraction on half of the detector rows, the
//                                rest mirrored by S(-q) = conj S(q));
//   NUMAG_PATH_SEPARABLE_BF16X3 / _BF16X6: every operand split into 2 or 3 bf16
//                                parts, 3 or 6 split products per real product on
//                                v_mfma_f32_16x16x32_bf16, FP32 accumulation.
// Twiddles are generated in FP64 into the workspace; the projection is a
// fixed-order FP64 sum.
//
// Loop mode (Sec. 3.1 loop modes, Sec. 3.2 data sets m_1 ... m_B): B weight
// snapshots on the same grid share the twiddles and run as 4 B channel sets
// through the same launches, so the contractions see B times the work per
// launch.  A snapshot's result does not depend on the others in the batch.
#include "numag_internal.h"
#include "phasor.h"

namespace numag {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Padded sizes of the operands, so that the matrix-core loads need no bounds
// checks: every padding entry is zero.
//   S  [sets][ny16][nzk]    projections (ny16 = ny rounded up to 32, nzk = nz to 16)
//   Ez [nzk][n1p]           column twiddles (n1p = n1 rounded up to 64)
//   T  [sets][ny16][n1p]    first contraction (complex)
//   Ey [n0p][nyk]           row twiddles (n0p = n0 to 32, nyk = ny to 16)
// nzk and nyk are the contraction depths, multiples of 16 so that the FP64
// kernels' loops (four or two K steps of 4 per iteration) need no remainder.
struct SepDims {
    int ny, nz, n0, n1, ny16, nzk, nyk, n0p, n1p;
};

struct SepLayout {
    size_t ey, ez, s, t, total;
};

// Paddings: rows of S and T (ny16) to the first contraction's 32-row wave tiles,
// detector rows and columns to 32 and 64 (the BF16 paths' tiles; the FP64 tiles
// are 16 x 16).
constexpr int kC1M = 32;
constexpr int kC2M = 32, kC2N = 64;
constexpr int kKStep = 16;  // padding of the contraction depths
// K steps of 4 per loop iteration of the first contraction (all their fragments
// loaded first, then the MFMAs).
constexpr int kC1Steps = 4;

__host__ __device__ static inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

static size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

static SepDims sep_dims(const numag_regular &g, const Detector &d)
{
    SepDims m{};
    m.ny = g.n[1];
    m.nz = g.n[2];
    m.n0 = d.n0;
    m.n1 = d.n1;
    m.ny16 = round_up(m.ny, kC1M);
    m.nzk = round_up(m.nz, kKStep);
    m.nyk = round_up(m.ny, kKStep);
    m.n0p = round_up(m.n0, kC2M);
    m.n1p = round_up(m.n1, kC2N);
    return m;
}

static SepLayout sep_layout(const numag_regular &g, const Detector &d, int64_t n_snap)
{
    const SepDims m = sep_dims(g, d);
    const size_t sets = 4 * (size_t)n_snap;
    SepLayout L{};
    L.ey = al((size_t)m.n0p * m.nyk * sizeof(double2));
    L.ez = al((size_t)m.nzk * m.n1p * sizeof(double2));
    L.s = al(sets * m.ny16 * m.nzk * sizeof(double));
    L.t = al(sets * m.ny16 * m.n1p * sizeof(double2));
    L.total = L.ey + L.ez + L.s + L.t;
    return L;
}

static size_t bf_bytes(const numag_regular &g, const Detector &d, int path, int64_t n_snap);

size_t separable_workspace_bytes(const numag_regular &g, const Detector &d, int path, int64_t n_snap)
{
    const SepLayout L = sep_layout(g, d, n_snap);
    if (path == NUMAG_PATH_SEPARABLE_F64 || path == NUMAG_PATH_SEPARABLE_F64_HERMITIAN) return L.total;
    // the BF16 paths also use the FP64 projections (the S region) before splitting them
    return L.s + bf_bytes(g, d, path, n_snap);
}

constexpr int kProjThreads = 64;  // columns per projection workgroup
constexpr int kProjSlices = 4;    // x slices per column (one thread each)
constexpr int kProjUnroll = 8;    // loads in flight per thread

// One launch for the operands of both contractions.
// Workgroups [0, n_proj * n_snap): projections (all paths).  Snapshot b's weights
// are two row-major matrices over x, nuc [nx][nyz] and mag [nx][3 nyz]; their
// column sums over x are the projections (column m of mag is component m % 3 of
// cell m / 3).  A workgroup owns 64 consecutive columns of the 4 nyz (nuc first,
// then mag), one per thread of a slice; x is split into 4 slices summed by 4
// threads in x order, the slices added in a fixed order through LDS.  Output
// S[4 b + c][iy][iz].
// The remaining workgroups: twiddles Ey[i][iy] = exp(-i q_y(i) y_iy) and
// Ez[iz][k] = exp(-i q_z(k) z_iz), zeros in the padding, and zeros in the
// padding of S.
// The weights are read once, with 8-byte non-temporal loads: measured on the
// 537 MB of 64 snapshots of a 64^3 grid in this layout, 77 us (7.0 TB/s) against
// 82 us with 16-byte loads of two adjacent columns per thread, and 88 us with
// ordinary loads; 2 or 8 slices, or 16 loads in flight, were no faster.
__device__ __forceinline__ double project_column(const double *__restrict__ src, int64_t stride, int nx, int slice)
{
    double acc = 0.0;
    int ix = slice;
    for (; ix + (kProjUnroll - 1) * kProjSlices < nx; ix += kProjUnroll * kProjSlices) {
        double v[kProjUnroll];
#pragma unroll
        for (int u = 0; u < kProjUnroll; ++u) v[u] = __builtin_nontemporal_load(src + (int64_t)(ix + u * kProjSlices) * stride);
#pragma unroll
        for (int u = 0; u < kProjUnroll; ++u) acc += v[u];
    }
    for (; ix < nx; ix += kProjSlices) acc += src[(int64_t)ix * stride];
    return acc;
}

__global__ __launch_bounds__(256) void sep_prepare_kernel(Detector d, numag_regular g, SepDims m,
                                                          const double *__restrict__ nuc,
                                                          const double *__restrict__ mag, int n_proj, int n_snap,
                                                          int tw, int pad_s, double *__restrict__ S,
                                                          double2 *__restrict__ ey, double2 *__restrict__ ez)
{
    const int64_t nyz = (int64_t)g.n[1] * g.n[2];
    const int64_t W = (int64_t)g.n[0] * nyz;
    const int64_t sstride = (int64_t)m.ny16 * m.nzk;  // one channel set of S
    if ((int64_t)blockIdx.x < (int64_t)n_proj * n_snap) {
        __shared__ double part[kProjSlices][kProjThreads];
        const int b = (int)(blockIdx.x / n_proj);
        const int col = threadIdx.x % kProjThreads, slice = threadIdx.x / kProjThreads;
        const int64_t mcol = (int64_t)(blockIdx.x % n_proj) * kProjThreads + col;  // in [0, 4 nyz)
        const bool is_nuc = mcol < nyz;
        const double *src = is_nuc ? (nuc != nullptr ? nuc + (int64_t)b * W + mcol : nullptr)
                                   : (mag != nullptr && mcol < 4 * nyz ? mag + (int64_t)b * W * 3 + (mcol - nyz)
                                                                       : nullptr);
        part[slice][col] = src != nullptr ? project_column(src, is_nuc ? nyz : 3 * nyz, g.n[0], slice) : 0.0;
        __syncthreads();
        // thread t < 64: column t of the workgroup, slices added in order
        const int t = threadIdx.x;
        const int64_t mc = (int64_t)(blockIdx.x % n_proj) * kProjThreads + t;
        if (t < kProjThreads && mc < 4 * nyz) {
            double v = 0.0;
            for (int sl = 0; sl < kProjSlices; ++sl) v += part[sl][t];
            const bool nc = mc < nyz;
            const int64_t cell = nc ? mc : (mc - nyz) / 3;
            const int c = nc ? 0 : 1 + (int)((mc - nyz) % 3);
            const int iy = (int)(cell / g.n[2]), iz = (int)(cell % g.n[2]);
            S[(int64_t)(4 * b + c) * sstride + (int64_t)iy * m.nzk + iz] = v;
        }
        return;
    }
    const int64_t idx = ((int64_t)blockIdx.x - (int64_t)n_proj * n_snap) * blockDim.x + threadIdx.x;
    // tw == 0: no FP64 twiddles (the BF16 paths write their own), padding of S only
    const int64_t ne = tw ? (int64_t)m.n0p * m.nyk : 0;
    const int64_t nez = tw ? (int64_t)m.nzk * m.n1p : 0;
    if (idx < ne) {
        const int i = (int)(idx / m.nyk), iy = (int)(idx % m.nyk);
        const double y = g.origin[1] + (double)iy * g.step[1];
        ey[idx] = (i < d.n0 && iy < m.ny) ? twiddle(axis_value(d.origin0, i, d.step0) * y) : make_double2(0.0, 0.0);
    } else if (idx < ne + nez) {
        const int64_t r = idx - ne;
        const int iz = (int)(r / m.n1p), k = (int)(r % m.n1p);
        const double z = g.origin[2] + (double)iz * g.step[2];
        ez[r] = (iz < m.nz && k < d.n1) ? twiddle(axis_value(d.origin1, k, d.step1) * z) : make_double2(0.0, 0.0);
    } else if (pad_s) {
        // padding of S: rows iy >= ny and columns iz >= nz of every channel set
        const int64_t r = idx - ne - nez;
        if (r < (int64_t)4 * n_snap * sstride) {
            const int64_t cell = r % sstride;
            const int iy = (int)(cell / m.nzk), iz = (int)(cell % m.nzk);
            if (iy >= m.ny || iz >= m.nz) S[r] = 0.0;
        }
    }
}

// ---- FP64 MFMA -------------------------------------------------------------
// Both contractions run on v_mfma_f64_16x16x4f64.  Lane layout: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16] of a K step of 4; accumulator register
// r holds D[4 r + l / 16][l % 16].  A wave owns 16 x 16 output tiles (MI x NI of
// them in the first contraction; in the second, one pixel tile of CSW channel
// sets).  Every output element takes the same instruction sequence whatever the
// tile shape or the channel sets a wave holds, so neither changes a result: a
// batch of snapshots gives each snapshot its single-call sums bit for bit.
// The 4 x 4 x 4 form issues its flops at a higher rate, but its register-blocked
// tiles need 2.5 times the operand loads per flop.  Measured on 64 snapshots
// (ny = nz = 64, 256 x 256 detector) against register-blocked 4 x 4 x 4 tiles:
// first contraction 41 -> 27 us, second 236 -> 181 us, bit-identical results.

// T[c][iy][k] = sum_iz S[c][iy][iz] Ez[iz][k] (real x complex: two products per
// step, into independent accumulators).
template <int MI, int NI>
__global__ __launch_bounds__(256) void sep_contract1_f64(const double *__restrict__ S, const double2 *__restrict__ Ez,
                                                         SepDims m, int n_sets, double2 *__restrict__ T)
{
    constexpr int TM = 16 * MI, TN = 16 * NI;
    const int lane = threadIdx.x & 63;
    const int tm = m.ny16 / TM, tn = m.n1p / TN;
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= (int64_t)n_sets * tm * tn) return;
    const int c = (int)(tile / ((int64_t)tm * tn));
    const int rem = (int)(tile % ((int64_t)tm * tn));
    const int i0 = (rem / tn) * TM, k0 = (rem % tn) * TN;
    const int r16 = lane & 15, kq = lane >> 4;
    const double *pa = S + (int64_t)c * m.ny16 * m.nzk + (int64_t)(i0 + r16) * m.nzk + kq;  // + 16 mi nzk + z0
    const double2 *pb = Ez + (int64_t)kq * m.n1p + k0 + r16;                                 // + z0 n1p + 16 ni
    v4d accR[MI][NI], accI[MI][NI];
#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < NI; ++ni) accR[mi][ni] = accI[mi][ni] = v4d{0.0, 0.0, 0.0, 0.0};
    auto load = [&](int z0, double (&a)[MI], double2 (&b)[NI]) {
#pragma unroll
        for (int mi = 0; mi < MI; ++mi) a[mi] = pa[(int64_t)16 * mi * m.nzk + z0];
#pragma unroll
        for (int ni = 0; ni < NI; ++ni) b[ni] = pb[(int64_t)z0 * m.n1p + 16 * ni];
    };
    auto mma = [&](const double (&a)[MI], const double2 (&b)[NI]) {
#pragma unroll
        for (int mi = 0; mi < MI; ++mi)
#pragma unroll
            for (int ni = 0; ni < NI; ++ni) {
                accR[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mi], b[ni].x, accR[mi][ni], 0, 0, 0);
                accI[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mi], b[ni].y, accI[mi][ni], 0, 0, 0);
            }
    };
    // kC1Steps K steps per iteration: all their fragments are loaded first, and the
    // MFMAs take them as they arrive
    for (int z0 = 0; z0 < m.nzk; z0 += 4 * kC1Steps) {
        double a[kC1Steps][MI];
        double2 b[kC1Steps][NI];
#pragma unroll
        for (int u = 0; u < kC1Steps; ++u) load(z0 + 4 * u, a[u], b[u]);
#pragma unroll
        for (int u = 0; u < kC1Steps; ++u) mma(a[u], b[u]);
    }
    double2 *Tc = T + (int64_t)c * m.ny16 * m.n1p;
#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < NI; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                Tc[(int64_t)(i0 + 16 * mi + 4 * r + kq) * m.n1p + k0 + 16 * ni + r16] =
                    make_double2(accR[mi][ni][r], accI[mi][ni][r]);
}

// F[c][i][k] = sum_iy Ey[i][iy] T[c][iy][k]  ->  amp[c / 4][(i n1 + k)][c % 4]
//
// This contraction carries nine tenths of the flops; the complex product is four
// real products per K step.  A wave owns one 16 x 16 pixel tile of CSW channel
// sets: CSW = 4 holds all four channel sets of a snapshot and shares the Ey
// fragment between them; CSW = 1 (four times the waves, for small batches) puts
// the four channel sets of a tile in the four waves of one workgroup, which write
// the same records together.  With CSW = 4 the result leaves through LDS: a lane
// holds four rows of one column, so a direct store instruction would scatter 16
// bytes into each of 64 pixel records; staged by rows, every store instruction
// writes 16 whole records (1 KB) of one row (170 against 190 us for 64 snapshots;
// 123 against 154 us on the Hermitian half).  Measured alternatives: larger
// register tiles (32 x 32, 32 x 64 pixels) lose occupancy and run slower, a
// deeper prefetch ring (four one-step buffers) gains without LDS stores but loses
// with them, a persistent grid-stride loop over tiles gains nothing, non-temporal
// stores of the result more than double the time, and the complex product as
// three real products (Gauss's trick, with the sums A + B and C + D as extra
// operand planes) cut the MFMA work by a quarter but added half again to the
// operand loads (1.5 times slower, with the earlier tiles).  A16: the result
// pointer is 16-byte aligned (one 16-byte store per channel).  HERM: only rows
// [0, ceil(n0 / 2)) are contracted, and each of their pixels p also writes the
// conjugate at the mirrored pixel P - 1 - p (S(-q) = conj S(q) for real weights
// on the symmetric Cartesian detector); the middle row of an odd n0 is contracted
// for every column and mirrors nothing.
template <int CSW, bool A16, bool HERM>
__global__ __launch_bounds__(256) void sep_contract2_f64(const double2 *__restrict__ Ey, const double2 *__restrict__ T,
                                                         SepDims m, int n_sets, double *__restrict__ amp)
{
    static_assert(CSW == 1 || CSW == 4, "one or four channel sets per wave");
    static_assert(kC2M % 16 == 0 && kC2N % 16 == 0, "tiles inside the padding");
    const int lane = threadIdx.x & 63;
    const int nr = HERM ? (m.n0 + 1) / 2 : m.n0;  // contracted rows
    const int tm = (nr + 15) / 16, tn = (m.n1 + 15) / 16;
    const int64_t tiles = (int64_t)tm * tn;
    // a wave past the last tile works on tile 0 and stores nothing (the LDS store
    // path has workgroup barriers)
    const int64_t tile_w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const bool active = tile_w < (int64_t)(n_sets / CSW) * tiles;
    const int64_t tile = active ? tile_w : 0;
    int64_t c0;
    int rem;
    if (CSW == 4) {
        c0 = 4 * (tile / tiles);
        rem = (int)(tile % tiles);
    } else {
        const int64_t r2 = tile % (4 * tiles);
        c0 = 4 * (tile / (4 * tiles)) + (r2 & 3);
        rem = (int)(r2 >> 2);
    }
    const int i0 = (rem / tn) * 16, k0 = (rem % tn) * 16;
    const int r16 = lane & 15, kq = lane >> 4;
    const int64_t cs = (int64_t)m.ny16 * m.n1p;  // one channel set of T
    // this lane's operand streams (every index stays inside the padded arrays)
    const double2 *pa = Ey + (int64_t)(i0 + r16) * m.nyk + kq;               // + y0
    const double2 *pb = T + c0 * cs + (int64_t)kq * m.n1p + k0 + r16;        // + ch cs + y0 n1p
    v4d accR[CSW], accI[CSW];
#pragma unroll
    for (int ch = 0; ch < CSW; ++ch) accR[ch] = accI[ch] = v4d{0.0, 0.0, 0.0, 0.0};
    auto load = [&](int y0, double2 &a, double2 (&b)[CSW]) {
        a = pa[y0];
#pragma unroll
        for (int ch = 0; ch < CSW; ++ch) b[ch] = pb[ch * cs + (int64_t)y0 * m.n1p];
    };
    // Two passes, so that the two products an accumulator takes per K step are issued
    // 2 CSW instructions apart (each accumulator takes them in the same order).
    auto mma = [&](const double2 &a, const double2 (&b)[CSW]) {
#pragma unroll
        for (int ch = 0; ch < CSW; ++ch) {
            accR[ch] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b[ch].x, accR[ch], 0, 0, 0);
            accI[ch] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b[ch].y, accI[ch], 0, 0, 0);
        }
#pragma unroll
        for (int ch = 0; ch < CSW; ++ch) {
            accR[ch] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b[ch].y, accR[ch], 0, 0, 0);
            accI[ch] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b[ch].x, accI[ch], 0, 0, 0);
        }
    };
    // Two register buffers of one K step each: the next step's fragments load while
    // this one's MFMAs run (three waves per SIMD).  nyk is a multiple of 8, so an
    // iteration takes two steps and needs no exit test; the last iteration's
    // prefetch reloads an in-bounds step.  Measured against loading two or four
    // steps and then running their MFMAs: 181 against 197 and 204 us.
    double2 a0, b0[CSW], a1, b1[CSW];
    load(0, a0, b0);
    for (int y0 = 0; y0 < m.nyk; y0 += 8) {
        load(y0 + 4, a1, b1);
        mma(a0, b0);
        load(min(y0 + 8, m.nyk - 4), a0, b0);
        mma(a1, b1);
    }
    const int col = k0 + r16;
    const int64_t P = (int64_t)m.n0 * m.n1;
    if (CSW == 4) {
        __shared__ double2 stage[4][4][16][4];  // [wave][row of the group][column][channel]
        const int w = threadIdx.x >> 6;
        const int px = lane >> 2, chl = lane & 3;  // the record part this lane stores
        double *dst = amp + (c0 >> 2) * P * 8 + 2 * chl;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int ch = 0; ch < CSW; ++ch) stage[w][kq][r16][ch] = make_double2(accR[ch][r], accI[ch][r]);
            __syncthreads();
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int row = i0 + 4 * r + s;
                if (!active || row >= nr) continue;
                if (k0 + px < m.n1) {
                    const double2 v = stage[w][s][px][chl];
                    double *o = dst + ((int64_t)row * m.n1 + k0 + px) * 8;
                    if (A16) {
                        *(double2 *)o = v;
                    } else {
                        o[0] = v.x;
                        o[1] = v.y;
                    }
                }
                // mirrored pixels of this row segment, P - 1 - p, ascending in px
                const int cm = k0 + 15 - px;
                if (HERM && row < m.n0 - nr && cm < m.n1) {
                    const double2 v = stage[w][s][15 - px][chl];
                    double *o = dst + (P - 1 - ((int64_t)row * m.n1 + cm)) * 8;
                    if (A16) {
                        *(double2 *)o = make_double2(v.x, -v.y);
                    } else {
                        o[0] = v.x;
                        o[1] = -v.y;
                    }
                }
            }
            __syncthreads();
        }
        return;
    }
    if (!active) return;
    double *dst = amp + (c0 >> 2) * P * 8 + 2 * (c0 & 3);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = i0 + 4 * r + kq;
        if (row >= nr || col >= m.n1) continue;
        const int64_t p = (int64_t)row * m.n1 + col;
        const bool mirror = HERM && row < m.n0 - nr;
        double *o = dst + p * 8;
        double *om = dst + (P - 1 - p) * 8;
        if (A16) {
            ((double2 *)o)[0] = make_double2(accR[0][r], accI[0][r]);
            if (mirror) ((double2 *)om)[0] = make_double2(accR[0][r], -accI[0][r]);
        } else {
            o[0] = accR[0][r];
            o[1] = accI[0][r];
            if (mirror) {
                om[0] = accR[0][r];
                om[1] = -accI[0][r];
            }
        }
    }
}

// ---- BF16 split products -------------------------------------------------
// NUMAG_PATH_SEPARABLE_BF16X3 / _BF16X6: every operand x is split into NP = 2 or 3
// bf16 parts (x = p0 + p1 [+ p2], each the bf16 rounding of what the previous
// parts leave, the remainders exact in FP64) and a real product takes the split
// pairs (i, j) with i + j < NP -- 3 or 6 products -- on v_mfma_f32_16x16x32_bf16,
// accumulated in FP32.  The parts are formed once, where an operand is written:
// the twiddles by the prepare kernel, the projections by the projection, the first
// contraction's result by that contraction, each into "K-contiguous" planes so
// that a lane reads its 8 consecutive K elements of a plane with one 16-byte load.
// Lane layout of the 16 x 16 x 32 form (one-hot probe): A[l % 16][8 (l / 16) + v],
// B[8 (l / 16) + v][l % 16] for v < 8, D[4 (l / 16) + r][l % 16].
//   Sb  [NP][sets][ny32][nz32]       projections, row y, K = z
//   EzT [NP][2][n1p][nz32]           column twiddles transposed (column k, K = z), re / im
//   Eyb [NP][2][n0p][ny32]           row twiddles (row i, K = y), re / im
//   TT  [NP][2][sets][n1p][ny32]     first contraction transposed (column k, K = y), re / im
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

struct BfLayout {
    int np, ny32, nz32;
    size_t s, ez, ey, t, total;
};

static BfLayout bf_layout(const SepDims &m, int path, int64_t n_snap)
{
    BfLayout L{};
    L.np = path == NUMAG_PATH_SEPARABLE_BF16X6 ? 3 : 2;
    L.ny32 = round_up(m.ny, 32);
    L.nz32 = round_up(m.nz, 32);
    const size_t sets = 4 * (size_t)n_snap, h = sizeof(unsigned short);
    L.s = al((size_t)L.np * sets * L.ny32 * L.nz32 * h);
    L.ez = al((size_t)L.np * 2 * m.n1p * L.nz32 * h);
    L.ey = al((size_t)L.np * 2 * m.n0p * L.ny32 * h);
    L.t = al((size_t)L.np * 2 * sets * m.n1p * L.ny32 * h);
    L.total = L.s + L.ez + L.ey + L.t;
    return L;
}

__device__ __forceinline__ unsigned short to_bf16(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ double from_bf16(unsigned short h) { return (double)__uint_as_float(((uint32_t)h) << 16); }

// The NP bf16 parts of x, written to dst[p * pstride].
template <int NP>
__device__ __forceinline__ void store_split(double x, unsigned short *dst, int64_t pstride)
{
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        const unsigned short h = to_bf16((float)x);
        dst[(int64_t)p * pstride] = h;
        x -= from_bf16(h);
    }
}

// Four consecutive K elements of one plane, split: the parts of v[0..3] packed as
// 4 bf16 per plane.
template <int NP>
__device__ __forceinline__ void store_split4(const float (&v)[4], unsigned short *dst, int64_t pstride)
{
    double r[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) r[j] = (double)v[j];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        unsigned short h[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            h[j] = to_bf16((float)r[j]);
            r[j] -= from_bf16(h[j]);
        }
        uint2 w;
        w.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
        w.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
        *(uint2 *)(dst + (int64_t)p * pstride) = w;
    }
}

__device__ __forceinline__ v8bf load8(const unsigned short *p) { return __builtin_bit_cast(v8bf, *(const uint4 *)p); }

// acc[q] += sum over the split pairs (i, j), i + j < NP, of a[q][i] b[q][j] for NQ
// independent products, the smallest split pairs first; the NQ accumulators take
// their instructions in turn, so consecutive instructions never depend on each
// other.
template <int NP, int NQ>
__device__ __forceinline__ void mfma_split(const v8bf (*const (&a)[NQ])[NP], const v8bf (*const (&b)[NQ])[NP],
                                           v4f (&acc)[NQ])
{
#pragma unroll
    for (int t = NP - 1; t >= 0; --t)
#pragma unroll
        for (int i = t; i >= 0; --i)
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16((*a[q])[i], (*b[q])[t - i], acc[q], 0, 0, 0);
}

// Twiddles and the padding of the projections of the BF16 paths (the projection
// itself is sep_prepare_kernel's, written split by sep_split_s_kernel).
template <int NP>
__global__ __launch_bounds__(256) void sep_twiddles_bf16(Detector d, numag_regular g, SepDims m, int ny32, int nz32,
                                                         unsigned short *__restrict__ eyb,
                                                         unsigned short *__restrict__ ezt)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ne = (int64_t)m.n0p * ny32;
    const int64_t nezt = (int64_t)m.n1p * nz32;
    if (idx < ne) {
        const int i = (int)(idx / ny32), iy = (int)(idx % ny32);
        const double y = g.origin[1] + (double)iy * g.step[1];
        const double2 e =
            (i < d.n0 && iy < m.ny) ? twiddle(axis_value(d.origin0, i, d.step0) * y) : make_double2(0.0, 0.0);
        store_split<NP>(e.x, eyb + idx, 2 * ne);
        store_split<NP>(e.y, eyb + ne + idx, 2 * ne);
    } else if (idx < ne + nezt) {
        const int64_t r = idx - ne;
        const int k = (int)(r / nz32), iz = (int)(r % nz32);
        const double z = g.origin[2] + (double)iz * g.step[2];
        const double2 e =
            (k < d.n1 && iz < m.nz) ? twiddle(axis_value(d.origin1, k, d.step1) * z) : make_double2(0.0, 0.0);
        store_split<NP>(e.x, ezt + r, 2 * nezt);
        store_split<NP>(e.y, ezt + nezt + r, 2 * nezt);
    }
}

// Split projections: Sb[p][set][iy][iz] from the FP64 S[set][ny16][nzk] (zero beyond ny, nz).
template <int NP>
__global__ __launch_bounds__(256) void sep_split_s_kernel(const double *__restrict__ S, SepDims m, int ny32,
                                                          int nz32, int sets, unsigned short *__restrict__ sb)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)ny32 * nz32;
    if (idx >= (int64_t)sets * per) return;
    const int set = (int)(idx / per);
    const int iy = (int)((idx % per) / nz32), iz = (int)(idx % nz32);
    const double v = (iy < m.ny && iz < m.nz) ? S[((int64_t)set * m.ny16 + iy) * m.nzk + iz] : 0.0;
    store_split<NP>(v, sb + idx, (int64_t)sets * per);
}

// T[c][y][k] = sum_z S[c][y][z] Ez[z][k] on 16 x 16 tiles, written split and
// transposed into TT[p][re / im][c][k][y].
template <int NP>
__global__ __launch_bounds__(256) void sep_contract1_bf16(const unsigned short *__restrict__ sb,
                                                          const unsigned short *__restrict__ ezt, SepDims m, int ny32,
                                                          int nz32, int sets, unsigned short *__restrict__ tt)
{
    const int lane = threadIdx.x & 63;
    const int tm = ny32 / 16, tn = m.n1p / 16;
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= (int64_t)sets * tm * tn) return;
    const int c = (int)(tile / ((int64_t)tm * tn));
    const int rem = (int)(tile % ((int64_t)tm * tn));
    const int m0 = (rem / tn) * 16, n0 = (rem % tn) * 16;
    const int kq = lane >> 4;
    const int64_t sp = (int64_t)sets * ny32 * nz32;  // part stride of Sb
    const int64_t ep = (int64_t)2 * m.n1p * nz32;    // part stride of EzT
    const unsigned short *pa = sb + ((int64_t)c * ny32 + m0 + (lane & 15)) * nz32 + 8 * kq;
    const unsigned short *pr = ezt + (int64_t)(n0 + (lane & 15)) * nz32 + 8 * kq;
    const unsigned short *pi = pr + (int64_t)m.n1p * nz32;
    v4f acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};  // re, im
    for (int k0 = 0; k0 < nz32; k0 += 32) {
        v8bf a[NP], br[NP], bi[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            a[p] = load8(pa + p * sp + k0);
            br[p] = load8(pr + p * ep + k0);
            bi[p] = load8(pi + p * ep + k0);
        }
        const v8bf (*const as[2])[NP] = {&a, &a};
        const v8bf (*const bs[2])[NP] = {&br, &bi};
        mfma_split<NP, 2>(as, bs, acc);
    }
    const v4f accR = acc[0], accI = acc[1];
    // D[4 kq + r][lane % 16]: rows y = m0 + 4 kq + r of column k = n0 + lane % 16
    const int64_t tp = (int64_t)2 * sets * m.n1p * ny32;  // part stride of TT
    unsigned short *dr = tt + ((int64_t)c * m.n1p + n0 + (lane & 15)) * ny32 + m0 + 4 * kq;
    unsigned short *di = dr + (int64_t)sets * m.n1p * ny32;
    const float vr[4] = {accR[0], accR[1], accR[2], accR[3]};
    const float vi[4] = {accI[0], accI[1], accI[2], accI[3]};
    store_split4<NP>(vr, dr, tp);
    store_split4<NP>(vi, di, tp);
}

// F[c][i][k] = sum_y Ey[i][y] T[c][y][k] on 16 x 16 tiles (four real products).
template <int NP>
__global__ __launch_bounds__(256) void sep_contract2_bf16(const unsigned short *__restrict__ eyb,
                                                          const unsigned short *__restrict__ tt, SepDims m, int ny32,
                                                          int sets, double *__restrict__ amp)
{
    const int lane = threadIdx.x & 63;
    const int tm = (m.n0 + 15) / 16, tn = (m.n1 + 15) / 16;
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= (int64_t)sets * tm * tn) return;
    const int c = (int)(tile / ((int64_t)tm * tn));
    const int rem = (int)(tile % ((int64_t)tm * tn));
    const int m0 = (rem / tn) * 16, n0 = (rem % tn) * 16;
    const int kq = lane >> 4;
    const int64_t ne = (int64_t)m.n0p * ny32;            // one re / im plane of Ey
    const int64_t nt = (int64_t)sets * m.n1p * ny32;     // one re / im plane of TT
    const unsigned short *par = eyb + (int64_t)(m0 + (lane & 15)) * ny32 + 8 * kq;
    const unsigned short *pai = par + ne;
    const unsigned short *pbr = tt + ((int64_t)c * m.n1p + n0 + (lane & 15)) * ny32 + 8 * kq;
    const unsigned short *pbi = pbr + nt;
    v4f acc[4] = {};  // Re A Re B, Im A Im B, Re A Im B, Im A Re B
    for (int y0 = 0; y0 < ny32; y0 += 32) {
        v8bf ar[NP], ai[NP], br[NP], bi[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            ar[p] = load8(par + p * 2 * ne + y0);
            ai[p] = load8(pai + p * 2 * ne + y0);
            br[p] = load8(pbr + p * 2 * nt + y0);
            bi[p] = load8(pbi + p * 2 * nt + y0);
        }
        const v8bf (*const as[4])[NP] = {&ar, &ai, &ar, &ai};
        const v8bf (*const bs[4])[NP] = {&br, &bi, &bi, &br};
        mfma_split<NP, 4>(as, bs, acc);
    }
    const v4f rr = acc[0], ii = acc[1], ri = acc[2], ir = acc[3];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = m0 + 4 * kq + r, k = n0 + (lane & 15);
        if (i < m.n0 && k < m.n1) {
            double *o = amp + (((int64_t)(c >> 2) * m.n0 + i) * m.n1 + k) * 8 + 2 * (c & 3);
            o[0] = (double)rr[r] - (double)ii[r];
            o[1] = (double)ri[r] + (double)ir[r];
        }
    }
}

template <int NP>
static int launch_bf16_path(const SepDims &m, const BfLayout &B, const Detector &d, const numag_regular &g,
                            const double *S, int sets, char *base, double *amp, hipStream_t s)
{
    unsigned short *sb = (unsigned short *)base;
    unsigned short *ezt = (unsigned short *)(base + B.s);
    unsigned short *eyb = (unsigned short *)(base + B.s + B.ez);
    unsigned short *tt = (unsigned short *)(base + B.s + B.ez + B.ey);
    const int64_t ntw = (int64_t)m.n0p * B.ny32 + (int64_t)m.n1p * B.nz32;
    hipLaunchKernelGGL((sep_twiddles_bf16<NP>), dim3((unsigned)((ntw + 255) / 256)), dim3(256), 0, s, d, g, m, B.ny32,
                       B.nz32, eyb, ezt);
    NUMAG_HIP_CHECK(hipGetLastError());
    const int64_t ns = (int64_t)sets * B.ny32 * B.nz32;
    hipLaunchKernelGGL((sep_split_s_kernel<NP>), dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, s, S, m, B.ny32,
                       B.nz32, sets, sb);
    NUMAG_HIP_CHECK(hipGetLastError());
    const int64_t t1 = (int64_t)sets * (B.ny32 / 16) * (m.n1p / 16);
    hipLaunchKernelGGL((sep_contract1_bf16<NP>), dim3((unsigned)((t1 + 3) / 4)), dim3(256), 0, s, sb, ezt, m, B.ny32,
                       B.nz32, sets, tt);
    NUMAG_HIP_CHECK(hipGetLastError());
    const int64_t t2 = (int64_t)sets * ((d.n0 + 15) / 16) * ((d.n1 + 15) / 16);
    hipLaunchKernelGGL((sep_contract2_bf16<NP>), dim3((unsigned)((t2 + 3) / 4)), dim3(256), 0, s, eyb, tt, m, B.ny32,
                       sets, amp);
    NUMAG_HIP_CHECK(hipGetLastError());
    return NUMAG_OK;
}

// FP64 path for snapshots [b0, b1): projection (+ twiddles when tw), then both
// contractions; every buffer offset by the first snapshot.
static int launch_f64_chunk(const double *nuc, const double *mag, const numag_regular &g, const Detector &d,
                            const SepDims &m, int64_t b0, int64_t b1, bool tw, bool herm, double2 *ey, double2 *ez,
                            double *S, double2 *T, double *amp, hipStream_t s)
{
    const int64_t W = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int64_t nb = b1 - b0;
    const int sets = (int)(4 * nb);
    const int64_t sstride = (int64_t)m.ny16 * m.nzk;
    if (nuc != nullptr) nuc += b0 * W;
    if (mag != nullptr) mag += b0 * W * 3;
    S += 4 * b0 * sstride;
    T += 4 * b0 * (int64_t)m.ny16 * m.n1p;
    amp += b0 * (int64_t)d.n0 * d.n1 * 8;
    const int64_t nyz = (int64_t)m.ny * m.nz;
    const int64_t n_proj = (4 * nyz + kProjThreads - 1) / kProjThreads;
    const bool pad_s = m.ny16 != m.ny || m.nzk != m.nz;
    const int64_t n_elem = (tw ? (int64_t)m.n0p * m.nyk + (int64_t)m.nzk * m.n1p : 0) +
                           (pad_s ? (int64_t)sets * sstride : 0);
    const int64_t n_tw = (n_elem + 255) / 256;
    hipLaunchKernelGGL(sep_prepare_kernel, dim3((unsigned)(n_proj * nb + n_tw)), dim3(256), 0, s, d, g, m, nuc, mag,
                       (int)n_proj, (int)nb, tw ? 1 : 0, pad_s ? 1 : 0, S, ey, ez);
    NUMAG_HIP_CHECK(hipGetLastError());
    // first contraction: 32 x 64 or 16 x 64 outputs per wave when that still makes
    // a few workgroups per CU, else 16 x 16
    const int64_t t1big = (int64_t)sets * (m.ny16 / 32) * (m.n1p / 64);
    const int64_t t1mid = (int64_t)sets * (m.ny16 / 16) * (m.n1p / 64);
    if (t1big >= 2048) {
        hipLaunchKernelGGL((sep_contract1_f64<2, 4>), dim3((unsigned)((t1big + 3) / 4)), dim3(256), 0, s, S, ez, m,
                           sets, T);
    } else if (t1mid >= 2048) {
        hipLaunchKernelGGL((sep_contract1_f64<1, 4>), dim3((unsigned)((t1mid + 3) / 4)), dim3(256), 0, s, S, ez, m,
                           sets, T);
    } else {
        const int64_t t1 = (int64_t)sets * (m.ny16 / 16) * (m.n1p / 16);
        hipLaunchKernelGGL((sep_contract1_f64<1, 1>), dim3((unsigned)((t1 + 3) / 4)), dim3(256), 0, s, S, ez, m, sets,
                           T);
    }
    NUMAG_HIP_CHECK(hipGetLastError());
    // second contraction: all four channel sets of a pixel tile in one wave when
    // that still makes 1024 workgroups, else one channel set per wave
    const int nr = herm ? (d.n0 + 1) / 2 : d.n0;  // contracted rows
    const int64_t t2 = nb * ((nr + 15) / 16) * ((d.n1 + 15) / 16);  // pixel tiles of all snapshots
    const bool a16 = ((uintptr_t)amp % 16) == 0;
    const unsigned g4 = (unsigned)((t2 + 3) / 4), g1 = (unsigned)t2;  // 4 waves per workgroup
#define NUMAG_LAUNCH_C2(CSW, A16, HERM, G) \
    hipLaunchKernelGGL((sep_contract2_f64<CSW, A16, HERM>), dim3(G), dim3(256), 0, s, ey, T, m, sets, amp)
    const int variant = (t2 >= 4096 ? 4 : 0) + (a16 ? 2 : 0) + (herm ? 1 : 0);
    switch (variant) {
        case 0: NUMAG_LAUNCH_C2(1, false, false, g1); break;
        case 1: NUMAG_LAUNCH_C2(1, false, true, g1); break;
        case 2: NUMAG_LAUNCH_C2(1, true, false, g1); break;
        case 3: NUMAG_LAUNCH_C2(1, true, true, g1); break;
        case 4: NUMAG_LAUNCH_C2(4, false, false, g4); break;
        case 5: NUMAG_LAUNCH_C2(4, false, true, g4); break;
        case 6: NUMAG_LAUNCH_C2(4, true, false, g4); break;
        default: NUMAG_LAUNCH_C2(4, true, true, g4); break;
    }
#undef NUMAG_LAUNCH_C2
    NUMAG_HIP_CHECK(hipGetLastError());
    return NUMAG_OK;
}

int launch_separable(const double *nuc, const double *mag, const numag_regular &g, const Detector &d, int path,
                     int64_t n_snap, double *amp, void *ws, size_t ws_bytes, hipStream_t s)
{
    const SepLayout L = sep_layout(g, d, n_snap);
    const SepDims m = sep_dims(g, d);
    const bool herm = path == NUMAG_PATH_SEPARABLE_F64_HERMITIAN;
    const bool f64 = path == NUMAG_PATH_SEPARABLE_F64 || herm;
    if (ws_bytes < separable_workspace_bytes(g, d, path, n_snap) || ws == nullptr) {
        set_error("numag_amplitudes: workspace too small for the separable path");
        return NUMAG_E_WORKSPACE;
    }
    const int64_t nyz = (int64_t)m.ny * m.nz;
    const bool pad_s = m.ny16 != m.ny || m.nzk != m.nz;
    if ((4 * nyz + kProjThreads - 1) / kProjThreads * n_snap +
            ((int64_t)m.n0p * m.nyk + (int64_t)m.nzk * m.n1p + (pad_s ? 4 * n_snap * m.ny16 * m.nzk : 0)) / 256 + 1 >
        0x7fffffffLL) {
        set_error("numag_amplitudes: too many snapshots for one separable call");
        return NUMAG_E_INVALID;
    }
    // FP64 path: Ey, Ez, S, T.  BF16 paths: S, then their split operands.
    char *base = (char *)ws;
    double2 *ey = f64 ? (double2 *)base : nullptr;
    double2 *ez = f64 ? (double2 *)(base + L.ey) : nullptr;
    double *S = (double *)(f64 ? base + L.ey + L.ez : base);
    double2 *T = f64 ? (double2 *)(base + L.ey + L.ez + L.s) : nullptr;
    if (!f64) {
        const int sets = (int)(4 * n_snap);
        const int64_t n_proj = (4 * nyz + kProjThreads - 1) / kProjThreads;
        const int64_t n_tw = ((pad_s ? (int64_t)sets * m.ny16 * m.nzk : 0) + 255) / 256;
        hipLaunchKernelGGL(sep_prepare_kernel, dim3((unsigned)(n_proj * n_snap + n_tw)), dim3(256), 0, s, d, g, m, nuc,
                           mag, (int)n_proj, (int)n_snap, 0, pad_s ? 1 : 0, S, nullptr, nullptr);
        NUMAG_HIP_CHECK(hipGetLastError());
        const BfLayout B = bf_layout(m, path, n_snap);
        char *bbase = base + L.s;
        return B.np == 3 ? launch_bf16_path<3>(m, B, d, g, S, sets, bbase, amp, s)
                         : launch_bf16_path<2>(m, B, d, g, S, sets, bbase, amp, s);
    }
    // One launch sequence for the whole batch.  Splitting the batch into chunks on two
    // streams, so that the projection (HBM-bound) of a chunk runs beside the second
    // contraction of the previous one, was measured slower for 64 snapshots: 0.30, 0.32
    // and 0.37 ms for 2, 4 and 8 chunks against 0.27-0.29 ms for one sequence (0.27
    // against 0.20 ms on the Hermitian half); the two kernels slow each other down more
    // than the overlap saves.
    return launch_f64_chunk(nuc, mag, g, d, m, 0, n_snap, true, herm, ey, ez, S, T, amp, s);
}

}  // namespace numag

namespace numag {
static size_t bf_bytes(const numag_regular &g, const Detector &d, int path, int64_t n_snap)
{
    return bf_layout(sep_dims(g, d), path, n_snap).total;
}
}  // namespace numag
