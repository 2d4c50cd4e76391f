// Small device helpers shared by the sum kernels: complex product, FP64 sine and
// cosine, the unit phasor exp(-i phi), and a detector axis value computed
// exactly as the detector is defined (one rounded product, one rounded sum,
// never fused).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/numag.h"
#include "types.h"

namespace numag {

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}


// sin x and cos x in FP64 for the sum kernels' generation phases.
// Cody-Waite reduction (Cody & Waite, Software Manual for the Elementary
// Functions, 1980): x = k pi/2 + r with pi/2 split into P1 + P2 + P3, P1 and P2
// holding 33 significant bits each, so k P1 and k P2 are exact for |k| < 2^20,
// and P3 the next 53 bits (the split reproduces pi/2 to 1e-37; derived from
// Machin's series for pi).  sin r and cos r on |r| <= pi/4 are the Taylor
// series through r^17 and r^16 (truncation below 0.05 ulp), evaluated by
// Horner's rule in r^2; the quadrant k mod 4 swaps and negates them.  Arguments
// beyond 2^19 take the library sincos.  Host-callable so that its accuracy can
// be checked without a GPU.
__host__ __device__ __forceinline__ void sincos_cw(double x, double *sp, double *cp)
{
    if (!(fabs(x) < 0x1p19)) {  // also NaN and infinities
        sincos(x, sp, cp);
        return;
    }
    constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
    constexpr double P1 = 0x1.921fb54400000p+0;
    constexpr double P2 = 0x1.0b4611a600000p-34;
    constexpr double P3 = 0x1.3198a2e037073p-69;
    const double k = rint(x * kTwoOverPi);
    const double r = fma(-k, P3, fma(-k, P2, fma(-k, P1, x)));
    const double z = r * r;
    // sin: r + r z (S3 + z (S5 + ... + z S17)),  S_n = (-1)^((n-1)/2) / n!
    double ps = 0x1.952c77030ad4ap-49;
    ps = fma(ps, z, -0x1.ae7f3e733b81fp-41);
    ps = fma(ps, z, 0x1.6124613a86d09p-33);
    ps = fma(ps, z, -0x1.ae64567f544e4p-26);
    ps = fma(ps, z, 0x1.71de3a556c734p-19);
    ps = fma(ps, z, -0x1.a01a01a01a01ap-13);
    ps = fma(ps, z, 0x1.1111111111111p-7);
    ps = fma(ps, z, -0x1.5555555555555p-3);
    const double sn = fma(r * z, ps, r);
    // cos: 1 + z (C2 + z (C4 + ... + z C16)),  C_n = (-1)^(n/2) / n!
    double pc = 0x1.ae7f3e733b81fp-45;
    pc = fma(pc, z, -0x1.93974a8c07c9dp-37);
    pc = fma(pc, z, 0x1.1eed8eff8d898p-29);
    pc = fma(pc, z, -0x1.27e4fb7789f5cp-22);
    pc = fma(pc, z, 0x1.a01a01a01a01ap-16);
    pc = fma(pc, z, -0x1.6c16c16c16c17p-10);
    pc = fma(pc, z, 0x1.5555555555555p-5);
    pc = fma(pc, z, -0x1.0000000000000p-1);
    const double cs = fma(z, pc, 1.0);
    // x = k pi/2 + r: quadrant n = k mod 4
    const int n = (int)k & 3;
    const double s0 = (n & 1) ? cs : sn;
    const double c0 = (n & 1) ? sn : cs;
    *sp = (n & 2) ? -s0 : s0;
    *cp = ((n + 1) & 2) ? -c0 : c0;
}

// exp(-i phi) = (cos phi, -sin phi)
__host__ __device__ __forceinline__ double2 twiddle(double phi)
{
    double s, c;
    sincos_cw(phi, &s, &c);
    return make_double2(c, -s);
}

// origin + i * step
__device__ __forceinline__ double axis_value(double origin, int i, double step)
{
#pragma clang fp contract(off)
    double t = (double)i * step;
    return origin + t;
}

// Unit vector of pixel p of a full detector (Cartesian: q / |q| with q = 0 -> e_z,
// |q| without fused operations; polar: the column angle, also at q = 0):
// qhat = (0, s, c).
__device__ __forceinline__ void pixel_qhat(const Detector &d, int64_t p, double &s, double &c)
{
    const int row = (int)(p / d.n1), col = (int)(p % d.n1);
    if (d.kind == NUMAG_GRID_CARTESIAN) {
        const double qy = axis_value(d.origin0, row, d.step0);
        const double qz = axis_value(d.origin1, col, d.step1);
        if (qy == 0.0 && qz == 0.0) {
            s = 0.0;
            c = 1.0;
            return;
        }
        double qn;
        {
#pragma clang fp contract(off)
            double a2 = qy * qy;
            double b2 = qz * qz;
            qn = sqrt(a2 + b2);
        }
        s = qy / qn;
        c = qz / qn;
    } else {
        const double th = (2.0 * 3.141592653589793 * (double)col) / (double)d.n_theta;
        sincos(th, &s, &c);
    }
}

}  // namespace numag
