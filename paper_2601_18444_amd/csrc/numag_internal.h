// Internal declarations of the numag HIP library (gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/numag.h"
#include "types.h"

namespace numag {

// ---------------------------------------------------------------------------
// Error reporting (thread-local message behind numag_last_error()).
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
void clear_error();

#define NUMAG_HIP_CHECK(expr)                                                        \
    do {                                                                             \
        hipError_t err_ = (expr);                                                    \
        if (err_ != hipSuccess) {                                                    \
            ::numag::set_error(std::string(#expr) + ": " + hipGetErrorString(err_)); \
            return NUMAG_E_HIP;                                                      \
        }                                                                            \
    } while (0)

// ---------------------------------------------------------------------------
// Kernel timer: TimedLaunch brackets one kernel launch with a HIP event pair
// on its stream while numag_kernel_timer is enabled.
// ---------------------------------------------------------------------------
bool timer_enabled();
int timer_begin(int kernel, hipStream_t s);   // returns a record id, or -1
void timer_end(int id, hipStream_t s);

struct TimedLaunch {
    int id;
    hipStream_t s;
    TimedLaunch(int kernel, hipStream_t st) : id(timer_enabled() ? timer_begin(kernel, st) : -1), s(st) {}
    ~TimedLaunch()
    {
        if (id >= 0) timer_end(id, s);
    }
};

Detector make_detector(const numag_qgrid &g);

// Validation of a numag_amplitudes request (sample, detector, rotations, path and
// mode); `fn` prefixes the error message.  NUMAG_OK or the status to return.
int validate_amplitudes_request(const numag_sample *sample, int64_t n_rot, const double *rot,
                                const numag_qgrid *grid, int32_t path, int32_t mode, const char *fn);

// ---------------------------------------------------------------------------
// Launchers (each enqueues on `stream`, returns NUMAG_OK or NUMAG_E_HIP).
// ---------------------------------------------------------------------------

// X_j = R (x_j + r^{k(j)}), w'_j = (n_j, R m_j) of the points j in [j_lo, j_hi),
// written to out[j - j_lo].  The object of a point follows from the HOST CSR
// offsets h_offsets [K+1] (read on the host and passed to the kernels by value,
// in groups of objects; unused when obj_pos is nullptr or K == 1).
int launch_prepare_points(const double *pos, const double *nuc, const double *mag, int64_t j_lo, int64_t j_hi,
                          const numag_regular *regular, const int64_t *h_offsets, int64_t K,
                          const double *obj_pos, const Rot &R, PointRec *out, hipStream_t s);

// direct Cartesian sum.  Writes [nsplit][P][8] partial sums (or the final
// [P][8] sums when nsplit == 1) for points [0, W).
struct DirectPlan {
    int lanes;       // lanes per detector row (Cartesian) or theta columns per workgroup (polar)
    int shape;       // polar: workgroup shape (index into the polar kernel's shapes)
    int channels;    // channels summed: 4 (N, M), 3 (M only) or 1 (N only); the rest are written as 0
    int nsplit;      // point ranges summed by different workgroups
    int64_t per;     // points per split (multiple of the chunk)
    int col_blocks, row_blocks;
};
// Hermitian completion of a half-detector sum (see direct.hip).
int launch_mirror_cartesian(double *amp, int64_t P, int64_t Ph, hipStream_t s);
// accumulate != 0: add into `out` instead of overwriting it
int launch_combine_polar_half(const double *part, int nsplit, int n0, int nh, double *out, hipStream_t s,
                              int accumulate = 0);

// Workgroups a direct-sum launch aims for (split-K included).
int target_workgroups();

// ---------------------------------------------------------------------------
// Launch-shape table (tune.hip): tuned shapes keyed by kernel, the evaluated
// detector and the point-count class; plans fall back to the defaults below.
// ---------------------------------------------------------------------------
enum { kTuneDirect = 0, kTuneAdjoint = 1, kTuneObjects = 2, kTuneKernelCount = 3 };
struct TuneShape {
    int shape;   // Cartesian direct / objects: lanes per row; polar direct: workgroup shape; adjoint: 0
    int target;  // workgroups (objects: work items) a launch aims for
};
int tune_wclass(int64_t W);
bool tuned_shape(int kernel, const Detector &d, int64_t W, TuneShape *out);
void tune_store(int kernel, const Detector &d, int64_t W, const TuneShape &s, double ms, double default_ms);
void tune_erase(int kernel, const Detector &d, int64_t W);
int tune_save();
void tune_clear();
bool valid_tune_shape(int kernel, const Detector &d, const TuneShape &s);
// The library's untuned shape for a kernel on detector d (evaluated part) and W points.
TuneShape default_tune_shape(int kernel, const Detector &d, int64_t W);
// The shape in use: the tuned one if the table holds it, else the default.
TuneShape current_tune_shape(int kernel, const Detector &d, int64_t W);
// max_splits > 0 caps the point splits (and so the partial-sum buffer).
DirectPlan plan_direct_cartesian(const Detector &d, int64_t W, int64_t max_splits = 0);
size_t direct_partial_bytes(const DirectPlan &p, const Detector &d);
int launch_direct_cartesian(const PointRec *pts, int64_t W, const Detector &d, const DirectPlan &p,
                            double *partial, hipStream_t s);

// Polar detector direct sum: [nsplit][P][8] partials.
// max_splits > 0 caps the point splits (rotation groups trade splits for rotations);
// shape >= 0 picks a workgroup shape (else the default for the detector) and
// target_wgs > 0 the workgroups aimed for (else the library default).
constexpr int kPolarShapeCount = 5;
int default_polar_shape(const Detector &d);
int polar_shape_rows(int shape);
int polar_shape_cols(int shape);
int polar_shape_waves(int shape);
DirectPlan plan_direct_polar(const Detector &d, int64_t W, int64_t max_splits = 0, int shape = -1,
                             int target_wgs = 0);
// n_rot > 1: pts holds n_rot consecutive copies of W points (one per rotation of a
// group) and the partials are [n_rot][p.nsplit][P][8].
int launch_direct_polar(const PointRec *pts, int64_t W, const Detector &d, const DirectPlan &p,
                        double *partial, hipStream_t s, int n_rot = 1);
// out[i] = value for i < n (a kernel, so that callers may capture it in a graph).
int launch_fill(double *out, int64_t n, double value, hipStream_t s);

// Fixed-order sum of split partials: out[p][v] = sum_s part[s][p][v] (v < 8),
// optionally added to `out` (accumulate != 0).
int launch_combine(const double *part, int nsplit, int64_t P, double *out, int accumulate,
                   hipStream_t s);

// work items (object slot, rotation group, pixel block); each sums complete
// objects and adds F F^H (and, in split mode, exp(-i q.R r^k) F) into an
// accumulator slot no other item touches; slots are reduced in a fixed order.
struct ObjectsPlan {
    int lanes;      // lanes per detector row
    int col_blocks, row_blocks;
    int n_slots;    // accumulator slots (object set x rotation range)
    int n_out;      // spectral matrices written (K per object, or 1)
    int64_t n_items;
};

// An object-mode (DILUTE / SPLIT) plan: everything the kernels need that depends
// on the host arguments (object offsets, rotations, work tables), as an image the
// caller uploads to the start of its workspace.  The image begins with a tag
// unique to the plan; the kernels compare it with the plan's and write NaN
// instead of reading tables that another plan, or other data, left there.
constexpr size_t kPlanTagBytes = 256;
struct ObjPlanTables;  // the persistent kernel's work tables (objects.hip)
struct ObjPlan {
    unsigned long long tag;
    Detector d;                 // the whole detector
    int path, mode, spec_per_object;
    int64_t n_rot, K, W;
    std::vector<int64_t> off;   // [K+1] host copy of the object offsets
    std::vector<char> image;    // uploaded to workspace offset 0: the tag, then the tables
    size_t o_rot = 0;           // rotations [n_rot][9] (doubles) within the image
    size_t ws_bytes = 0;        // workspace bytes the plan's calls need
    std::shared_ptr<ObjPlanTables> tables;  // the persistent kernel's tables
};
// Detector part the object kernel sums: all of d, or with `hermitian` the first
// ceil(n0 / 2) rows of a Cartesian detector or the theta columns [0, n_theta / 2)
// of a polar one (the rest follow by G(-q) = conj G(q)).
Detector objects_detector(const Detector &d, bool hermitian);
// Fills pl.tables, pl.image (rotations excepted), pl.o_rot and pl.ws_bytes of a plan
// whose other fields are set (either detector kind).
void build_objects_plan(ObjPlan &pl);
// out[i] = NaN (i < n) when the tag at tag_ptr is not `tag`.
int launch_tag_guard(const unsigned long long *tag_ptr, unsigned long long tag, double *out, int64_t n,
                     hipStream_t st);
// Enqueues the sums of a plan whose image is in `ws` (kernels only).
int launch_objects_plan(const ObjPlan &pl, const numag_sample &s, double *spec_out, double *amp_out, void *ws,
                        hipStream_t st);

// cross sections from amplitudes ([n_sets][P][8]) or spectra ([n_sets][P][16]).
int launch_cross_section(const Detector &d, int64_t n_sets, const double *amp, const double *spec,
                         const numag_consts &c, uint32_t mask, double *out, hipStream_t s);
// spec = scale A A^H per set and pixel (accumulate: spec += scale A A^H)
int launch_spectral_matrix(int64_t n_sets, int64_t P, const double *amp, double *spec, hipStream_t s,
                           double scale = 1.0, int accumulate = 0);

// a8
int launch_azimuthal(const Detector &d, const double *f, int n_f, int n_bins, double qmax_avg,
                     double *I, int64_t *count, hipStream_t s);

// a9
int launch_correlation(const double *q, const double *I, int n_q, int n_f, const double *r, int n_r,
                       double scale, double *c, double *p, hipStream_t s);

// residual weights, loss, adjoint sum (hermitian: over half of a detector that
// is symmetric about q = 0, with the residual weights folded onto it).
int launch_grad(const PointRec *pts, int64_t W, const Detector &d, const numag_consts &c,
                const double *amp, const double *target, const double *weight, double *loss,
                double *dnuc, double *dmag, const Rot &R, void *ws, size_t ws_bytes, hipStream_t s,
                bool hermitian = false);
// Workspace bytes of launch_grad on detector d (whole), for the path it will run.
size_t grad_workspace_bytes(const Detector &d, int64_t W, bool hermitian);

// 2D correlation function (eq. crav2d) from data on detector d onto real-space grid rd.
size_t correlation_2d_workspace_bytes(const Detector &d, const Detector &rd);
int launch_correlation_2d(const Detector &d, const double *f, int n_f, const Detector &rd, double *C, void *ws,
                          size_t ws_bytes, hipStream_t s);

// Angular spectrum (eqs. CosineSinceIntensities, ModalAmplitudes) on a polar detector.
int launch_angular_spectrum(const Detector &d, const double *f, int n_f, int k_max, double *Is, double *Ic,
                            double *As, double *Ac, hipStream_t s);

// regular-grid separable path on the matrix cores, for n_snap weight snapshots
// (nuc [n_snap][W], mag [n_snap][W][3]; amp [n_snap][P][8]).
int launch_separable(const double *nuc, const double *mag, const numag_regular &g, const Detector &d,
                     int path, int64_t n_snap, double *amp, void *ws, size_t ws_bytes, hipStream_t s);
size_t separable_workspace_bytes(const numag_regular &g, const Detector &d, int path, int64_t n_snap);

}  // namespace numag
