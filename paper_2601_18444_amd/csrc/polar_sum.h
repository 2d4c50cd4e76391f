// Device building block of the polar-detector sums (Sec. 3.2 (q, theta) grid),
// shared by the direct kernel (polar.hip) and the persistent object kernel
// (objects.hip).
//
// S_c(q_i, theta_m) = sum_j w_{j,c} exp(-i q_i u_m(j)),  u_m = Y sin(theta_m) + Z cos(theta_m).
// The phase does not separate, but along q it is a geometric sequence: a lane
// owns one theta column and walks 8 q rows, the first from its row group's start
// phasor, the second by one step exp(-i dq u), the rest by the two-term recurrence
// p_{r+1} = 2 cos(dq u) p_r - p_{r-1}.
//
// Workgroup shapes: WV waves, CW theta columns; a wave covers its CW columns with
// 64 / CW row groups of 8 rows, so the workgroup covers ROWS = 8 WV 64 / CW q rows.
// The per-(point, column) generation -- u, one sincos for the step, the block
// start exp(-i q(row0) u) as a power of the step, the row groups' starts by the
// same recurrence in step^8 -- is done once per workgroup and shared by its ROWS
// rows: narrower column blocks share it over more rows (and do fewer generations
// per workgroup) at the price of padding on detectors with fewer rows.
#pragma once

#include "cartesian_sum.h"

namespace numag {
namespace polar {

constexpr int kB = 8;  // q rows per lane

// The workgroup shapes the launchers instantiate (index = DirectPlan::shape).
struct ShapeDesc {
    int waves, cols, chunk, buffers;
};
constexpr ShapeDesc kShapes[kPolarShapeCount] = {
    {8, 64, 8, 2},   // 0: 64 rows x 64 columns, double-buffered chunks of 8 points
    {4, 64, 8, 1},   // 1: 32 rows x 64 columns (detectors of at most 32 q rows), two per CU
    {8, 32, 8, 2},   // 2: 128 rows x 32 columns, double-buffered
    {8, 16, 16, 1},  // 3: 256 rows x 16 columns, single-buffered chunks of 16 points
    {8, 16, 8, 2},   // 4: 256 rows x 16 columns, double-buffered chunks of 8 points
};

// Compile-time constants of one shape.
template <int WV, int CW, int CHK, int NB>
struct Shape {
    static_assert(CW == 64 || CW == 32 || CW == 16, "columns per workgroup");
    static constexpr int NT = 64 * WV;        // threads
    static constexpr int LPC = 64 / CW;       // row groups per wave
    static constexpr int G = WV * LPC;        // row groups per workgroup
    static constexpr int ROWS = kB * G;
    static constexpr int GEN = CHK * CW;      // (point, column) generations per chunk
    static constexpr int GPT = (GEN + NT - 1) / NT;  // generations per thread
    // one row per point of a chunk; single-buffered, plus one the pipelined loop
    // may read past the end (double-buffered, that read is clamped instead)
    static constexpr int R = NB == 2 ? CHK : CHK + 1;
    static_assert(GEN % 64 == 0, "generation is wave-uniform");
    static_assert(4 * CHK <= NT, "one weight component per thread");
};

template <int WV, int CW, int CHK, int NB>
struct Smem {
    using S = Shape<WV, CW, CHK, NB>;
    double2 start[NB][S::R][S::G][CW];  // start phasor of each row group and column
    double2 step[NB][S::R][CW];         // q step of each column
    double w[NB][S::R][4];
    double2 trig[CW];                   // (sin, cos) of the column angles
};

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

// This lane's theta column (within the block) and row group.
template <int WV, int CW>
__device__ __forceinline__ int lane_col() { return (threadIdx.x & 63) % CW; }
template <int WV, int CW>
__device__ __forceinline__ int lane_group() { return (threadIdx.x >> 6) * (64 / CW) + (threadIdx.x & 63) / CW; }

// Adds the points [jbeg, jend) of `ld` (cart::PointPart load(j, slot): lab-frame
// Y, Z and weight component `slot`) into acc for the block of columns
// [col0, col0 + CW) and rows [rb ROWS, (rb + 1) ROWS): the lane's 8 rows
// rb ROWS + 8 lane_group() + r of column col0 + lane_col().  Starts with a
// barrier and ends with one, so the shared buffers may be reused by the next call.
template <int WV, int CW, int CHK, int NB, int CH, class Loader>
__device__ __forceinline__ void accumulate(const Loader &ld, int64_t jbeg, int64_t jend, const Detector &d, int col0,
                                           int rb, Smem<WV, CW, CHK, NB> &sm, double (&acc)[kB][2 * CH])
{
    using S = Shape<WV, CW, CHK, NB>;
    constexpr int NT = S::NT, G = S::G, GEN = S::GEN, GPT = S::GPT;
    const int t = threadIdx.x;
    __syncthreads();  // a previous call may still read the buffers
    if (t < CW) {
        const double theta = (2.0 * 3.141592653589793 * (double)(col0 + t)) / (double)d.n_theta;
        double sth, cth;
        sincos(theta, &sth, &cth);
        sm.trig[t] = make_double2(sth, cth);
    }
    __syncthreads();
    const double qrow0 = axis_value(d.origin0, rb * S::ROWS, d.step0);

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
            nY[i] = 0.0;
            nZ[i] = 0.0;
            if (e < GEN && j < jend) {
                const cart::PointPart p = ld.load(j, 0);
                nY[i] = p.Y;
                nZ[i] = p.Z;
            }
        }
        nW = (wj < CHK && j1 + wj < jend) ? ld.load(j1 + wj, wc).w : 0.0;
    };
    // twiddles of the fetched chunk into LDS buffer b (zeros past the end)
    auto generate = [&](int b) {
#pragma unroll
        for (int i = 0; i < GPT; ++i) {
            const int e = t + NT * i;
            if (e >= GEN) break;  // wave-uniform
            const int jj = e / CW, c = e % CW;
            const double2 tr = sm.trig[c];
            const double u = nY[i] * tr.x + nZ[i] * tr.y;
            const double2 step = twiddle(d.step0 * u);
            double2 sb = cmul(step, step);  // step^8: from one row group to the next
            sb = cmul(sb, sb);
            sb = cmul(sb, sb);
            // start of the block exp(-i q(row0) u): with q rows from zero it is
            // step^row0 = (step^ROWS)^rb by binary powering (uniform over the
            // workgroup; the rounding of dq u is carried row0 times, a few times the
            // error of a sincos of q(row0) u, and each squaring adds one rounding)
            double2 st;
            if (d.origin0 == 0.0) {
                double2 base = sb;
#pragma unroll
                for (int g = 1; g < G; g += g) base = cmul(base, base);
                st = make_double2(1.0, 0.0);
                for (unsigned ex = (unsigned)rb; ex != 0; ex >>= 1) {
                    if (ex & 1) st = cmul(st, base);
                    if (ex > 1) base = cmul(base, base);
                }
            } else {
                st = twiddle(qrow0 * u);
            }
            sm.step[b][jj][c] = step;
            // row-group starts st sb^g by the two-term recurrence in g (G - 1 steps:
            // the error grows at most linearly in g)
            const double k8 = sb.x + sb.x;
            double2 pm = st, pc = cmul(st, sb);
            sm.start[b][jj][0][c] = pm;
            sm.start[b][jj][1][c] = pc;
#pragma unroll
            for (int g = 2; g < G; ++g) {
                const double2 pn = make_double2(fma(k8, pc.x, -pm.x), fma(k8, pc.y, -pm.y));
                sm.start[b][jj][g][c] = pn;
                pm = pc;
                pc = pn;
            }
        }
        if (wj < CHK) sm.w[b][wj][wc] = nW;
    };
    const int lc = lane_col<WV, CW>();
    const int lg = lane_group<WV, CW>();
    auto operands = [&](int b, int jj) {
        cart::Operands o;
        o.ez = sm.start[b][jj][lg][lc];
        o.dz = sm.step[b][jj][lc];
        o.k = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) o.w[v] = sm.w[b][jj][v];
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
            polar_point<kB, CH>(opa, acc);
            __builtin_amdgcn_sched_barrier(0);
            const int nxt = NB == 2 ? min(jj + 2, CHK - 1) : jj + 2;  // past the end: discarded
            opa = operands(b, nxt);
            __builtin_amdgcn_sched_barrier(0);
            polar_point<kB, CH>(opb, acc);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (jj < nk) polar_point<kB, CH>(opa, acc);
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
        __syncthreads();
    }
}

}  // namespace polar
}  // namespace numag
