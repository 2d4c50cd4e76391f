// Plain types the kernels take as arguments or read from device memory: the
// detector descriptor, a rotation, and the per-point record of the direct sums.
#pragma once

#include <cstdint>

namespace numag {

// ---------------------------------------------------------------------------
// Detector descriptor passed by value to kernels.
// q(i) = -qmax + i * step on both Cartesian axes (step = 2 qmax / (n - 1));
// polar: q(i) = i * step with step = qmax / (n_q - 1), theta_m = m * dtheta.
// ---------------------------------------------------------------------------
struct Detector {
    int kind;
    int n0, n1;            // rows and columns evaluated
    int n_theta;           // polar: columns of the full detector (theta_m = 2 pi m / n_theta)
    double qmax;
    double step0, step1;   // Cartesian: axis steps (rows, cols); polar: q step, theta step
    double origin0, origin1;
};


// Row-major 3x3 rotation as a kernel argument.
struct Rot {
    double m[9];
};

// Per-point record written by the preparation kernel: lab-frame Y, Z (q has
// no x component) and lab-frame weights (n, m'x, m'y, m'z), padded to 64 bytes.
struct alignas(64) PointRec {
    double Y, Z;
    double w[4];
    double pad[2];
};

}  // namespace numag
