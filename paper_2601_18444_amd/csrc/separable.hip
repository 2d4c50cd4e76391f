// Regular-grid separable path (matrix cores).  Placeholder until the kernels land.
#include "numag_internal.h"

namespace numag {

size_t separable_workspace_bytes(const numag_regular &g, const Detector &d, int path)
{
    (void)g;
    (void)d;
    (void)path;
    return 0;
}

int launch_separable(const double *nuc, const double *mag, const numag_regular &g, const Detector &d, int path,
                     double *amp, void *ws, size_t ws_bytes, hipStream_t s)
{
    (void)nuc; (void)mag; (void)g; (void)d; (void)path; (void)amp; (void)ws; (void)ws_bytes; (void)s;
    set_error("numag_amplitudes: separable path not available in this build");
    return NUMAG_E_UNSUPPORTED;
}

}  // namespace numag
