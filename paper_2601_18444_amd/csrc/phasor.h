// Small device helpers shared by the sum kernels: complex product, the unit
// phasor exp(-i phi), and a detector axis value computed exactly as the
// detector is defined (one rounded product, one rounded sum, never fused).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/numag.h"
#include "types.h"

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
