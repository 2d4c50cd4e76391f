// Host build of the sum kernels' FP64 sincos (sincos_cw): reads arguments as
// hexadecimal doubles on stdin, one per line, and prints "sin cos" of each as
// hexadecimal doubles.  Built and driven by tests/test_sincos_cw.py.
#include <cstdio>

#include "phasor.h"

int main()
{
    double x;
    while (std::scanf("%la", &x) == 1) {
        double s, c;
        numag::sincos_cw(x, &s, &c);
        std::printf("%a %a\n", s, c);
    }
    return 0;
}
