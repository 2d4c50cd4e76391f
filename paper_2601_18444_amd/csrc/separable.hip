// Regular-grid separable path on the gfx950 matrix cores.
//
// For points on a regular grid (micromagnetic cells) with no sample rotation,
// the lab phase q.r = q_y y + q_z z does not involve x, so the DSFT of Sec. 3.3
// factors exactly:
//   S_c(y, z)   = sum_x w_c(x, y, z)                      (projection along the beam)
//   T_c(y, k)   = sum_z S_c(y, z) exp(-i q_z(k) z)         (real x complex contraction)
//   F_c(i, k)   = sum_y exp(-i q_y(i) y) T_c(y, k)         (complex x complex contraction)
// The two contractions are dense GEMMs and run on MFMA:
//   NUMAG_PATH_SEPARABLE_F64:    FP64 operands and accumulation, the first on
//                                v_mfma_f64_16x16x4f64 (one wave per 16 x 16 tile),
//                                the second on v_mfma_f64_4x4x4f64 (register-blocked
//                                16 x 16 or 32 x 32 tiles, see sep_contract2_f64);
//   NUMAG_PATH_SEPARABLE_BF16X3: v_mfma_f32_16x16x16bf16_1k with every operand split
//                                into bf16 hi + lo and the three products hi*hi,
//                                hi*lo, lo*hi accumulated in FP32.
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
typedef short v4s __attribute__((ext_vector_type(4)));

struct SepLayout {
    size_t ey, ez, s, t, total;
};

// Output tile of one wave in the second contraction (rows i, columns k).
constexpr int kC2M = 32, kC2N = 64;

// The operands of the second contraction are zero-padded so that its loads need
// no bounds checks: E_y is [n0p][nyp], T is [sets][nyp][n1p] with n0p, nyp, n1p
// the detector rows, grid y cells and detector columns rounded up to 32, 4, 64.
__host__ __device__ static inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

static size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

static SepLayout sep_layout(const numag_regular &g, const Detector &d, int64_t n_snap)
{
    const size_t ny = g.n[1], nz = g.n[2], n1 = d.n1, sets = 4 * (size_t)n_snap;
    const size_t n0p = round_up(d.n0, kC2M), nyp = round_up(g.n[1], 4), n1p = round_up(d.n1, kC2N);
    SepLayout L{};
    L.ey = al(n0p * nyp * sizeof(double2));
    L.ez = al(nz * n1 * sizeof(double2));
    L.s = al(sets * ny * nz * sizeof(double));
    L.t = al(sets * nyp * n1p * sizeof(double2));
    L.total = L.ey + L.ez + L.s + L.t;
    return L;
}

size_t separable_workspace_bytes(const numag_regular &g, const Detector &d, int path, int64_t n_snap)
{
    (void)path;
    return sep_layout(g, d, n_snap).total;
}

constexpr int kProjCells = 64;   // (y, z) cells per projection workgroup
constexpr int kProjSlices = 4;   // x slices per cell (one thread each)

// Sum over the x cells ix = slice, slice + kProjSlices, ... of column rem (a cell
// (iy, iz)), in x order.  Loads of four x cells are issued before their adds so
// that several are in flight (the projection is HBM-bound).
template <bool HN, bool HM>
__device__ __forceinline__ void project_cells(const double *__restrict__ nuc, const double *__restrict__ mag,
                                              int64_t rem, int64_t nyz, int nx, int slice, double (&s)[4])
{
    constexpr int U = 4;
    int ix = slice;
    for (; ix + (U - 1) * kProjSlices < nx; ix += U * kProjSlices) {
        double vn[U], vm[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t j = (int64_t)(ix + u * kProjSlices) * nyz + rem;
            vn[u] = HN ? nuc[j] : 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) vm[u][a] = HM ? mag[3 * j + a] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            s[0] += vn[u];
#pragma unroll
            for (int a = 0; a < 3; ++a) s[1 + a] += vm[u][a];
        }
    }
    for (; ix < nx; ix += kProjSlices) {
        const int64_t j = (int64_t)ix * nyz + rem;
        if (HN) s[0] += nuc[j];
        if (HM) {
#pragma unroll
            for (int a = 0; a < 3; ++a) s[1 + a] += mag[3 * j + a];
        }
    }
}

// One launch for the operands of both contractions.
// Workgroups [0, n_proj * n_snap): projection S[b][c][iy][iz] = sum_x w_c(x, iy, iz)
// of snapshot b for 64 cells, x split into 4 slices summed by 4 threads, slices
// added in a fixed order through LDS.  The remaining workgroups: twiddles
// Ey[i][iy] = exp(-i q_y(i) y_iy) and Ez[iz][k] = exp(-i q_z(k) z_iz).
__global__ __launch_bounds__(256) void sep_prepare_kernel(Detector d, numag_regular g, const double *__restrict__ nuc,
                                                          const double *__restrict__ mag, int n_proj, int n_snap,
                                                          double *__restrict__ S, double2 *__restrict__ ey,
                                                          double2 *__restrict__ ez)
{
    const int64_t nyz = (int64_t)g.n[1] * g.n[2];
    const int64_t W = (int64_t)g.n[0] * nyz;
    if ((int64_t)blockIdx.x < (int64_t)n_proj * n_snap) {
        __shared__ double part[kProjSlices][4][kProjCells];
        const int b = (int)(blockIdx.x / n_proj);
        if (nuc != nullptr) nuc += (int64_t)b * W;
        if (mag != nullptr) mag += (int64_t)b * W * 3;
        S += (int64_t)b * 4 * nyz;
        const int cell = threadIdx.x % kProjCells, slice = threadIdx.x / kProjCells;
        const int64_t rem = (int64_t)(blockIdx.x % n_proj) * kProjCells + cell;
        double s[4] = {0.0, 0.0, 0.0, 0.0};
        if (rem < nyz) {
            if (nuc != nullptr && mag != nullptr)
                project_cells<true, true>(nuc, mag, rem, nyz, g.n[0], slice, s);
            else if (mag != nullptr)
                project_cells<false, true>(nuc, mag, rem, nyz, g.n[0], slice, s);
            else if (nuc != nullptr)
                project_cells<true, false>(nuc, mag, rem, nyz, g.n[0], slice, s);
        }
        for (int c = 0; c < 4; ++c) part[slice][c][cell] = s[c];
        __syncthreads();
        // thread (c, cell) adds the slices in order
        const int c = threadIdx.x / kProjCells;
        if (rem < nyz) {
            double t = 0.0;
            for (int sl = 0; sl < kProjSlices; ++sl) t += part[sl][c][cell];
            S[c * nyz + rem] = t;
        }
        return;
    }
    const int64_t idx = ((int64_t)blockIdx.x - (int64_t)n_proj * n_snap) * blockDim.x + threadIdx.x;
    const int64_t ny = g.n[1], nz = g.n[2];
    const int64_t nyp = round_up(g.n[1], 4);
    const int64_t ne = (int64_t)round_up(d.n0, kC2M) * nyp;
    if (idx < ne) {
        const int i = (int)(idx / nyp), iy = (int)(idx % nyp);
        const double y = g.origin[1] + (double)iy * g.step[1];
        ey[idx] = (i < d.n0 && iy < ny) ? twiddle(axis_value(d.origin0, i, d.step0) * y) : make_double2(0.0, 0.0);
    } else if (idx < ne + nz * d.n1) {
        const int64_t r = idx - ne;
        const int iz = (int)(r / d.n1), k = (int)(r % d.n1);
        const double z = g.origin[2] + (double)iz * g.step[2];
        ez[r] = twiddle(axis_value(d.origin1, k, d.step1) * z);
    }
}

// ---- FP64 MFMA -------------------------------------------------------------
// v_mfma_f64_16x16x4f64 lane layout: A[l % 16][l / 16], B[l / 16][l % 16],
// D[4 r + l / 16][l % 16] for r < 4 (unlike the FP32-accumulating MFMAs below).

// T[c][iy][k] = sum_iz S[c][iy][iz] Ez[iz][k]
__global__ __launch_bounds__(256) void sep_contract1_f64(const double *__restrict__ S, const double2 *__restrict__ Ez,
                                                         int ny, int nz, int n1, int nyp, int n1p, int n_sets,
                                                         double2 *__restrict__ T)
{
    const int lane = threadIdx.x & 63;
    const int tm = (nyp + 15) / 16, tn = (n1p + 15) / 16;
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= (int64_t)n_sets * tm * tn) return;
    const int c = (int)(tile / (tm * tn));
    const int rem = (int)(tile % (tm * tn));
    const int m0 = (rem / tn) * 16, n0 = (rem % tn) * 16;
    const int ai = m0 + (lane & 15), bj = n0 + (lane & 15), kq = lane >> 4;
    const double *Sc = S + (int64_t)c * ny * nz;
    v4d accR = {0.0, 0.0, 0.0, 0.0}, accI = {0.0, 0.0, 0.0, 0.0};
    auto load = [&](int k, double &a, double2 &b) {
        const int kk = k + kq;
        a = (ai < ny && kk < nz) ? Sc[(int64_t)ai * nz + kk] : 0.0;
        b = (bj < n1 && kk < nz) ? Ez[(int64_t)kk * n1 + bj] : make_double2(0.0, 0.0);
    };
    // four K steps at a time: their loads are issued before their MFMAs (the
    // accumulation order is the same as one step at a time)
    constexpr int U = 4;
    int k = 0;
    for (; k + 4 * (U - 1) < nz; k += 4 * U) {
        double a[U];
        double2 b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) load(k + 4 * u, a[u], b[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            accR = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u].x, accR, 0, 0, 0);
            accI = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u].y, accI, 0, 0, 0);
        }
    }
    for (; k < nz; k += 4) {
        double a;
        double2 b;
        load(k, a, b);
        accR = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b.x, accR, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b.y, accI, 0, 0, 0);
    }
    double2 *Tc = T + (int64_t)c * nyp * n1p;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = m0 + 4 * r + kq;
        if (i < nyp && bj < n1p) Tc[(int64_t)i * n1p + bj] = make_double2(accR[r], accI[r]);
    }
}

// F[c][i][k] = sum_iy Ey[i][iy] T[c][iy][k]  ->  amp[c / 4][(i n1 + k)][c % 4]
//
// This contraction carries nine tenths of the flops, so it runs on
// v_mfma_f64_4x4x4f64 (four 4 x 4 x 4 blocks per instruction), which issues its
// flops faster on gfx950 than the 16 x 16 x 4 form.  Lane layout (one-hot probe):
// block g = (l / 4) % 4, A[g][l % 4][l / 16], B[g][l / 16][l % 4], D[g][l / 16][l % 4].
// A wave owns a (16 MG) x (4 NG) output tile: per K step of 4 it holds MG A
// fragments (rows i0 + 16 mg + 4 g + m) and NG B fragments (columns k0 + 4 ng + n,
// the same for every block) and issues MG x NG x 4 instructions (the complex
// product as four real ones).  Every output element sees the same instruction
// sequence whatever the tile shape, so the shape (chosen by the amount of work)
// does not change the result.
template <int MG, int NG>
__global__ __launch_bounds__(256) void sep_contract2_f64(const double2 *__restrict__ Ey, const double2 *__restrict__ T,
                                                         int n0, int n1, int nyp, int n1p, int n_sets,
                                                         double *__restrict__ amp)
{
    constexpr int TM = 16 * MG, TN = 4 * NG;
    static_assert(kC2M % TM == 0 && kC2N % TN == 0, "tile inside the padding");
    const int lane = threadIdx.x & 63;
    const int tm = (n0 + TM - 1) / TM, tn = (n1 + TN - 1) / TN;
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= (int64_t)n_sets * tm * tn) return;
    const int c = (int)(tile / ((int64_t)tm * tn));
    const int rem = (int)(tile % ((int64_t)tm * tn));
    const int i0 = (rem / tn) * TM, k0 = (rem % tn) * TN;
    const int g = (lane >> 2) & 3, e = lane & 3, kq = lane >> 4;
    // this lane's operand streams (every index stays inside the padded arrays)
    const double2 *pa = Ey + (int64_t)(i0 + 4 * g + e) * nyp + kq;               // + 16 mg nyp + y0
    const double2 *pb = T + (int64_t)c * nyp * n1p + (int64_t)kq * n1p + k0 + e;  // + y0 n1p + 4 ng
    double accR[MG][NG], accI[MG][NG];
#pragma unroll
    for (int mg = 0; mg < MG; ++mg)
#pragma unroll
        for (int ng = 0; ng < NG; ++ng) accR[mg][ng] = accI[mg][ng] = 0.0;

    auto load = [&](int y0, double2 (&a)[MG], double2 (&b)[NG]) {
#pragma unroll
        for (int mg = 0; mg < MG; ++mg) a[mg] = pa[(int64_t)16 * mg * nyp + y0];
#pragma unroll
        for (int ng = 0; ng < NG; ++ng) b[ng] = pb[(int64_t)y0 * n1p + 4 * ng];
    };
    auto mma = [&](const double2 (&a)[MG], const double2 (&b)[NG]) {
#pragma unroll
        for (int ng = 0; ng < NG; ++ng)
#pragma unroll
            for (int mg = 0; mg < MG; ++mg) {
                accR[mg][ng] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[mg].x, b[ng].x, accR[mg][ng], 0, 0, 0);
                accR[mg][ng] = __builtin_amdgcn_mfma_f64_4x4x4f64(-a[mg].y, b[ng].y, accR[mg][ng], 0, 0, 0);
                accI[mg][ng] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[mg].x, b[ng].y, accI[mg][ng], 0, 0, 0);
                accI[mg][ng] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[mg].y, b[ng].x, accI[mg][ng], 0, 0, 0);
            }
    };
    // two register buffers: the next K step's fragments load while this one's MFMAs run
    double2 a0[MG], b0[NG], a1[MG], b1[NG];
    load(0, a0, b0);
    for (int y0 = 0; y0 < nyp; y0 += 8) {
        const bool more = y0 + 4 < nyp;
        if (more) load(y0 + 4, a1, b1);
        mma(a0, b0);
        if (!more) break;
        if (y0 + 8 < nyp) load(y0 + 8, a0, b0);
        mma(a1, b1);
    }
    double *dst = amp + (int64_t)(c >> 2) * n0 * n1 * 8 + 2 * (c & 3);
#pragma unroll
    for (int mg = 0; mg < MG; ++mg) {
        const int row = i0 + 16 * mg + 4 * g + kq;
        if (row >= n0) continue;
#pragma unroll
        for (int ng = 0; ng < NG; ++ng) {
            const int col = k0 + 4 * ng + e;
            if (col < n1) {
                double *o = dst + ((int64_t)row * n1 + col) * 8;
                o[0] = accR[mg][ng];
                o[1] = accI[mg][ng];
            }
        }
    }
}

// ---- BF16 x 3 MFMA ---------------------------------------------------------
// v_mfma_f32_16x16x16bf16_1k lane layout: A[l % 16][4 (l / 16) + v],
// B[4 (l / 16) + v][l % 16] for v < 4, D[4 (l / 16) + r][l % 16].

__device__ __forceinline__ short to_bf16(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (short)(u >> 16);
}

__device__ __forceinline__ float from_bf16(short h) { return __uint_as_float(((uint32_t)(uint16_t)h) << 16); }

struct Bf3 {
    v4s hi, lo;
};

// element v of o: x = hi + lo, both bf16
__device__ __forceinline__ void split_bf16(double x, Bf3 &o, int v)
{
    const short hi = to_bf16((float)x);
    o.hi[v] = hi;
    o.lo[v] = to_bf16((float)(x - (double)from_bf16(hi)));
}

__device__ __forceinline__ v4f mfma3(const Bf3 &a, const Bf3 &b, v4f acc)
{
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.hi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.lo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.lo, b.hi, acc, 0, 0, 0);
    return acc;
}

__global__ __launch_bounds__(256) void sep_contract1_bf16x3(const double *__restrict__ S,
                                                            const double2 *__restrict__ Ez, int ny, int nz,
                                                            int n1, int nyp, int n1p, int n_sets,
                                                            double2 *__restrict__ T)
{
    const int lane = threadIdx.x & 63;
    const int tm = (nyp + 15) / 16, tn = (n1p + 15) / 16;
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= (int64_t)n_sets * tm * tn) return;
    const int c = (int)(tile / (tm * tn));
    const int rem = (int)(tile % (tm * tn));
    const int m0 = (rem / tn) * 16, n0 = (rem % tn) * 16;
    const int ai = m0 + (lane & 15), bj = n0 + (lane & 15), kq = lane >> 4;
    const double *Sc = S + (int64_t)c * ny * nz;
    v4f accR = {0.f, 0.f, 0.f, 0.f}, accI = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < nz; k += 16) {
        Bf3 a, br, bi;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int kk = k + 4 * kq + v;
            const double av = (ai < ny && kk < nz) ? Sc[(int64_t)ai * nz + kk] : 0.0;
            const double2 bv = (bj < n1 && kk < nz) ? Ez[(int64_t)kk * n1 + bj] : make_double2(0.0, 0.0);
            split_bf16(av, a, v);
            split_bf16(bv.x, br, v);
            split_bf16(bv.y, bi, v);
        }
        accR = mfma3(a, br, accR);
        accI = mfma3(a, bi, accI);
    }
    double2 *Tc = T + (int64_t)c * nyp * n1p;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = m0 + 4 * kq + r;
        if (i < nyp && bj < n1p) Tc[(int64_t)i * n1p + bj] = make_double2((double)accR[r], (double)accI[r]);
    }
}

__global__ __launch_bounds__(256) void sep_contract2_bf16x3(const double2 *__restrict__ Ey,
                                                            const double2 *__restrict__ T, int n0, int ny,
                                                            int n1, int nyp, int n1p, int n_sets,
                                                            double *__restrict__ amp)
{
    const int lane = threadIdx.x & 63;
    const int tm = (n0 + 15) / 16, tn = (n1 + 15) / 16;
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= (int64_t)n_sets * tm * tn) return;
    const int c = (int)(tile / (tm * tn));
    const int rem = (int)(tile % (tm * tn));
    const int m0 = (rem / tn) * 16, n0t = (rem % tn) * 16;
    const int ai = m0 + (lane & 15), bj = n0t + (lane & 15), kq = lane >> 4;
    const double2 *Tc = T + (int64_t)c * nyp * n1p;
    v4f accR = {0.f, 0.f, 0.f, 0.f}, accI = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < ny; k += 16) {
        Bf3 ar, ai_neg, aim, br, bi;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int kk = k + 4 * kq + v;
            const double2 av = (ai < n0 && kk < ny) ? Ey[(int64_t)ai * nyp + kk] : make_double2(0.0, 0.0);
            const double2 bv = (bj < n1 && kk < ny) ? Tc[(int64_t)kk * n1p + bj] : make_double2(0.0, 0.0);
            split_bf16(av.x, ar, v);
            split_bf16(av.y, aim, v);
            split_bf16(-av.y, ai_neg, v);
            split_bf16(bv.x, br, v);
            split_bf16(bv.y, bi, v);
        }
        accR = mfma3(ar, br, accR);
        accR = mfma3(ai_neg, bi, accR);
        accI = mfma3(ar, bi, accI);
        accI = mfma3(aim, br, accI);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = m0 + 4 * kq + r;
        if (i < n0 && bj < n1) {
            double *o = amp + (((int64_t)(c >> 2) * n0 + i) * n1 + bj) * 8 + 2 * (c & 3);
            o[0] = (double)accR[r];
            o[1] = (double)accI[r];
        }
    }
}

int launch_separable(const double *nuc, const double *mag, const numag_regular &g, const Detector &d, int path,
                     int64_t n_snap, double *amp, void *ws, size_t ws_bytes, hipStream_t s)
{
    const SepLayout L = sep_layout(g, d, n_snap);
    if (ws_bytes < L.total || ws == nullptr) {
        set_error("numag_amplitudes: workspace too small for the separable path");
        return NUMAG_E_WORKSPACE;
    }
    char *base = (char *)ws;
    double2 *ey = (double2 *)base;
    double2 *ez = (double2 *)(base + L.ey);
    double *S = (double *)(base + L.ey + L.ez);
    double2 *T = (double2 *)(base + L.ey + L.ez + L.s);
    const int ny = g.n[1], nz = g.n[2];
    const int nyp = round_up(ny, 4), n1p = round_up(d.n1, kC2N), n0p = round_up(d.n0, kC2M);
    const int sets = (int)(4 * n_snap);
    const int64_t ntw = (int64_t)n0p * nyp + (int64_t)nz * d.n1;
    const int64_t n_proj = ((int64_t)ny * nz + kProjCells - 1) / kProjCells;
    const int64_t n_tw = (ntw + 255) / 256;
    hipLaunchKernelGGL(sep_prepare_kernel, dim3((unsigned)(n_proj * n_snap + n_tw)), dim3(256), 0, s, d, g, nuc, mag,
                       (int)n_proj, (int)n_snap, S, ey, ez);
    NUMAG_HIP_CHECK(hipGetLastError());
    const int64_t t1 = (int64_t)sets * ((nyp + 15) / 16) * ((n1p + 15) / 16);
    const int64_t t2 = (int64_t)sets * ((d.n0 + 15) / 16) * ((d.n1 + 15) / 16);
    // 32 x 32 tiles when they give every SIMD a few waves, else 16 x 16
    const int64_t t2big = (int64_t)sets * ((d.n0 + 31) / 32) * ((d.n1 + 31) / 32);
    const bool big = t2big >= 4096;
    const int64_t t2f = big ? t2big : (int64_t)sets * ((d.n0 + 15) / 16) * ((d.n1 + 15) / 16);
    if (path == NUMAG_PATH_SEPARABLE_F64) {
        hipLaunchKernelGGL(sep_contract1_f64, dim3((unsigned)((t1 + 3) / 4)), dim3(256), 0, s, S, ez, ny, nz, d.n1,
                           nyp, n1p, sets, T);
        NUMAG_HIP_CHECK(hipGetLastError());
        if (big)
            hipLaunchKernelGGL((sep_contract2_f64<2, 8>), dim3((unsigned)((t2f + 3) / 4)), dim3(256), 0, s, ey, T,
                               d.n0, d.n1, nyp, n1p, sets, amp);
        else
            hipLaunchKernelGGL((sep_contract2_f64<1, 4>), dim3((unsigned)((t2f + 3) / 4)), dim3(256), 0, s, ey, T,
                               d.n0, d.n1, nyp, n1p, sets, amp);
    } else {
        hipLaunchKernelGGL(sep_contract1_bf16x3, dim3((unsigned)((t1 + 3) / 4)), dim3(256), 0, s, S, ez, ny, nz,
                           d.n1, nyp, n1p, sets, T);
        NUMAG_HIP_CHECK(hipGetLastError());
        hipLaunchKernelGGL(sep_contract2_bf16x3, dim3((unsigned)((t2 + 3) / 4)), dim3(256), 0, s, ey, T, d.n0, ny,
                           d.n1, nyp, n1p, sets, amp);
    }
    NUMAG_HIP_CHECK(hipGetLastError());
    return NUMAG_OK;
}

}  // namespace numag
