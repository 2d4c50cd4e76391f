// Small device helpers shared by the sum kernels: complex product, the unit
// phasor exp(-i phi), and a detector axis value computed exactly as the
// detector is defined (one rounded product, one rounded sum, never fused).
#pragma once

#include <hip/hip_runtime.h>

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

}  // namespace numag
