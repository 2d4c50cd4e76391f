// Allocation-free coherent direct sums (numag_amplitudes_noalloc): the COHERENT
// direct path of numag_amplitudes with its scratch -- the lab-frame point records
// and the split partial sums -- in one static device array instead of a caller
// workspace.
//
// In host code `scratch` names a host-side stand-in for the array, not its device
// address: the address is looked up once per device with hipGetSymbolAddress and
// only that address is handed to kernels.  The array keeps whatever the last call
// on its device left; every byte a call reads is written earlier in the same call
// (point records by the preparation kernel, partial sums by the sum kernel), so
// nothing needs clearing.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "numag_internal.h"

static __device__ __align__(256) unsigned char scratch[NUMAG_NOALLOC_SCRATCH_BYTES];

namespace numag {
namespace {

constexpr size_t kCap = NUMAG_NOALLOC_SCRATCH_BYTES;
constexpr size_t kPixelBytes = 8 * sizeof(double);  // one pixel of partial sums

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

std::mutex g_mu;
std::vector<void *> g_addr;  // device address of `scratch`, per device (nullptr: not looked up yet)

// Device address of the array on device `dev`, looked up with that device current.
int scratch_address(int dev, void **out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if ((size_t)dev < g_addr.size() && g_addr[dev] != nullptr) {
        *out = g_addr[dev];
        return NUMAG_OK;
    }
    int cur = 0;
    NUMAG_HIP_CHECK(hipGetDevice(&cur));
    if (cur != dev) NUMAG_HIP_CHECK(hipSetDevice(dev));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) NUMAG_HIP_CHECK(hipSetDevice(cur));
    if (e != hipSuccess || p == nullptr) {
        set_error(std::string("numag_amplitudes_noalloc: hipGetSymbolAddress of the static scratch failed: ") +
                  hipGetErrorString(e));
        return NUMAG_E_HIP;
    }
    if ((size_t)dev >= g_addr.size()) g_addr.resize((size_t)dev + 1, nullptr);
    g_addr[dev] = p;
    *out = p;
    return NUMAG_OK;
}

// Device on which work enqueued on `st` runs.
int stream_device(hipStream_t st, int *dev)
{
    if (st == nullptr) {
        NUMAG_HIP_CHECK(hipGetDevice(dev));
        return NUMAG_OK;
    }
    hipDevice_t d = 0;
    NUMAG_HIP_CHECK(hipStreamGetDevice(st, &d));
    *dev = (int)d;
    return NUMAG_OK;
}

// Pixels whose partial sums one launch writes: the whole detector, or the half
// that the Hermitian path evaluates.
Detector evaluated(const Detector &d, bool hermitian)
{
    Detector dh = d;
    if (hermitian) {
        if (d.kind == NUMAG_GRID_CARTESIAN) dh.n0 = (d.n0 + 1) / 2;
        else dh.n1 = d.n1 / 2;
    }
    return dh;
}

// The sums of one rotation with the scratch at `scr` (kCap bytes): the points go
// through in chunks as large as the space left after the partial sums allows;
// chunk c > 0 adds its combined partials into `amp`.
int run_bounded(const numag_sample &s, const Rot &R, const Detector &d, bool hermitian, double *amp, char *scr,
                hipStream_t st)
{
    const int64_t P = (int64_t)d.n0 * d.n1;
    const int64_t W = s.n_points;
    if (W == 0 || (s.nuc == nullptr && s.mag == nullptr)) return launch_fill(amp, P * 8, 0.0, st);
    const int channels = s.nuc == nullptr ? 3 : (s.mag == nullptr ? 1 : 4);
    const Detector dh = evaluated(d, hermitian);
    const int64_t Ph = (int64_t)dh.n0 * dh.n1;
    // splits: as the workspace path plans them, capped so the partial sums fill
    // at most half of the array; the rest holds a chunk of point records
    const int64_t max_splits = std::max<int64_t>(1, (int64_t)((kCap / 2) / ((size_t)Ph * kPixelBytes)));
    const bool cart = d.kind == NUMAG_GRID_CARTESIAN;
    DirectPlan p0 = cart ? plan_direct_cartesian(dh, W, max_splits) : plan_direct_polar(dh, W, max_splits);
    const size_t part_bytes = align256((size_t)p0.nsplit * (size_t)Ph * kPixelBytes);
    double *part = (double *)scr;
    PointRec *pts = (PointRec *)(scr + part_bytes);
    int64_t chunk = (int64_t)((kCap - part_bytes) / sizeof(PointRec));
    chunk -= chunk % 64;
    const int64_t n_chunks = (W + chunk - 1) / chunk;
    int rc = NUMAG_OK;
    for (int64_t c = 0; c < n_chunks && rc == NUMAG_OK; ++c) {
        const int64_t j0 = c * chunk, j1 = std::min(W, j0 + chunk), Wc = j1 - j0;
        rc = launch_prepare_points(s.pos, s.nuc, s.mag, j0, j1, s.regular, s.obj_offsets, s.n_objects, s.obj_pos, R,
                                   pts, st);
        if (rc != NUMAG_OK) break;
        // a chunk's plan has no more splits than the first chunk's (Wc <= W)
        DirectPlan p = n_chunks == 1 ? p0 : (cart ? plan_direct_cartesian(dh, Wc, p0.nsplit)
                                                  : plan_direct_polar(dh, Wc, p0.nsplit));
        p.channels = channels;
        const int acc = c > 0 ? 1 : 0;
        if (cart) {
            if (p.nsplit == 1 && n_chunks == 1) {
                rc = launch_direct_cartesian(pts, Wc, dh, p, amp, st);
            } else {
                rc = launch_direct_cartesian(pts, Wc, dh, p, part, st);
                if (rc == NUMAG_OK) rc = launch_combine(part, p.nsplit, Ph, amp, acc, st);
            }
        } else {
            rc = launch_direct_polar(pts, Wc, dh, p, part, st);
            if (rc == NUMAG_OK) {
                rc = hermitian ? launch_combine_polar_half(part, p.nsplit, d.n0, dh.n1, amp, st, acc)
                               : launch_combine(part, p.nsplit, Ph, amp, acc, st);
            }
        }
    }
    if (rc != NUMAG_OK || !hermitian || !cart) return rc;
    return launch_mirror_cartesian(amp, P, Ph, st);
}

}  // namespace
}  // namespace numag

using namespace numag;

extern "C" int numag_amplitudes_noalloc(const numag_sample *sample, int64_t n_rot, const double *rot,
                                        const numag_qgrid *grid, int32_t path, double *amp_out, void *stream)
{
    clear_error();
    if (path != NUMAG_PATH_DIRECT && path != NUMAG_PATH_DIRECT_HERMITIAN) {
        set_error("numag_amplitudes_noalloc: path must be NUMAG_PATH_DIRECT or NUMAG_PATH_DIRECT_HERMITIAN");
        return NUMAG_E_INVALID;
    }
    // the same validation as numag_amplitudes in COHERENT mode
    const int vrc = validate_amplitudes_request(sample, n_rot, rot, grid, path, NUMAG_MODE_COHERENT,
                                                "numag_amplitudes_noalloc");
    if (vrc != NUMAG_OK) return vrc;
    if (amp_out == nullptr) {
        set_error("numag_amplitudes_noalloc: amp_out is NULL");
        return NUMAG_E_INVALID;
    }
    const Detector d = make_detector(*grid);
    const bool hermitian = path == NUMAG_PATH_DIRECT_HERMITIAN;
    const Detector dh = evaluated(d, hermitian);
    const size_t need = (size_t)dh.n0 * (size_t)dh.n1 * kPixelBytes;
    if (need > kCap / 2) {
        set_error("numag_amplitudes_noalloc: the detector's partial sums need " + std::to_string(need) +
                  " bytes, more than half of the " + std::to_string(kCap) +
                  "-byte static scratch (at most " + std::to_string(kCap / 2 / kPixelBytes) +
                  " evaluated pixels); use numag_amplitudes with a workspace");
        return NUMAG_E_UNSUPPORTED;
    }
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    int rc = stream_device(st, &dev);
    if (rc != NUMAG_OK) return rc;
    void *scr = nullptr;
    if ((rc = scratch_address(dev, &scr)) != NUMAG_OK) return rc;
    const int64_t P = (int64_t)d.n0 * d.n1;
    for (int64_t r = 0; r < n_rot; ++r) {
        Rot R{};
        if (rot == nullptr) {
            R.m[0] = R.m[4] = R.m[8] = 1.0;
        } else {
            std::memcpy(R.m, rot + 9 * r, sizeof(R.m));
        }
        rc = run_bounded(*sample, R, d, hermitian, amp_out + r * P * 8, (char *)scr, st);
        if (rc != NUMAG_OK) return rc;
    }
    return NUMAG_OK;
}
