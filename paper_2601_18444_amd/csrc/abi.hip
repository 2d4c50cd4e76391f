// C ABI of the numag library: argument validation, workspace layout and dispatch.
// Host code only; every numerical step runs in the HIP kernels of this library.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <random>
#include <string>
#include <vector>

#include "numag_internal.h"

namespace numag {

static thread_local std::string g_error;

void set_error(const std::string &msg) { g_error = msg; }
void clear_error() { g_error.clear(); }

}  // namespace numag

using namespace numag;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

struct Carve {
    char *base;
    size_t used = 0;
    explicit Carve(void *p) : base((char *)p) {}
    void *take(size_t bytes)
    {
        void *r = base != nullptr ? base + used : nullptr;
        used += align_up(bytes);
        return r;
    }
};

bool is_separable(int32_t path)
{
    return path == NUMAG_PATH_SEPARABLE_F64 || path == NUMAG_PATH_SEPARABLE_BF16X3 ||
           path == NUMAG_PATH_SEPARABLE_BF16X6 || path == NUMAG_PATH_SEPARABLE_F64_HERMITIAN;
}

int invalid(const std::string &msg)
{
    set_error(msg);
    return NUMAG_E_INVALID;
}

bool is_finite(double x) { return std::isfinite(x); }

int check_grid(const numag_qgrid *g, const char *fn)
{
    if (g == nullptr) return invalid(std::string(fn) + ": grid is NULL");
    if (g->kind != NUMAG_GRID_CARTESIAN && g->kind != NUMAG_GRID_POLAR)
        return invalid(std::string(fn) + ": unknown detector kind");
    if (g->n0 < 1 || g->n1 < 1) return invalid(std::string(fn) + ": detector sizes must be >= 1");
    if ((int64_t)g->n0 * (int64_t)g->n1 > (int64_t)1 << 30)
        return invalid(std::string(fn) + ": detector larger than 2^30 pixels");
    if (!(g->qmax > 0.0) || !is_finite(g->qmax)) return invalid(std::string(fn) + ": qmax must be finite and > 0");
    return NUMAG_OK;
}

int check_sample(const numag_sample *s, const char *fn)
{
    if (s == nullptr) return invalid(std::string(fn) + ": sample is NULL");
    if (s->n_points < 0) return invalid(std::string(fn) + ": n_points < 0");
    if (s->n_objects < 1) return invalid(std::string(fn) + ": n_objects must be >= 1");
    if (s->regular != nullptr) {
        const numag_regular &g = *s->regular;
        if (g.n[0] < 1 || g.n[1] < 1 || g.n[2] < 1)
            return invalid(std::string(fn) + ": regular grid sizes must be >= 1");
        if ((int64_t)g.n[0] * g.n[1] * g.n[2] != s->n_points)
            return invalid(std::string(fn) + ": regular grid size does not match n_points");
        for (int a = 0; a < 3; ++a)
            if (!is_finite(g.origin[a]) || !is_finite(g.step[a]))
                return invalid(std::string(fn) + ": regular grid origin/step not finite");
    } else if (s->n_points > 0 && s->pos == nullptr) {
        return invalid(std::string(fn) + ": pos is NULL");
    }
    if (s->n_objects > 1) {
        if (s->obj_offsets == nullptr) return invalid(std::string(fn) + ": obj_offsets required when K > 1");
        const int64_t *o = s->obj_offsets;
        if (o[0] != 0 || o[s->n_objects] != s->n_points)
            return invalid(std::string(fn) + ": obj_offsets must start at 0 and end at n_points");
        for (int64_t k = 0; k < s->n_objects; ++k)
            if (o[k + 1] < o[k]) return invalid(std::string(fn) + ": obj_offsets not non-decreasing");
    }
    return NUMAG_OK;
}

int check_rotations(const double *rot, int64_t n_rot, const char *fn)
{
    if (n_rot < 1) return invalid(std::string(fn) + ": n_rot must be >= 1");
    if (rot == nullptr) {
        if (n_rot != 1) return invalid(std::string(fn) + ": rot NULL requires n_rot == 1");
        return NUMAG_OK;
    }
    for (int64_t r = 0; r < n_rot; ++r) {
        const double *R = rot + 9 * r;
        for (int a = 0; a < 9; ++a)
            if (!is_finite(R[a])) return invalid(std::string(fn) + ": rotation has non-finite entries");
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double dot = R[3 * a] * R[3 * b] + R[3 * a + 1] * R[3 * b + 1] + R[3 * a + 2] * R[3 * b + 2];
                if (std::fabs(dot - (a == b ? 1.0 : 0.0)) > 1e-9)
                    return invalid(std::string(fn) + ": rotation matrix is not orthonormal");
            }
        double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                     R[2] * (R[3] * R[7] - R[4] * R[6]);
        if (det < 0.0) return invalid(std::string(fn) + ": rotation matrix has det -1");
    }
    return NUMAG_OK;
}

Rot rot_of(const double *rot, int64_t r)
{
    Rot R{};
    if (rot == nullptr) {
        R.m[0] = R.m[4] = R.m[8] = 1.0;
    } else {
        std::memcpy(R.m, rot + 9 * r, sizeof(R.m));
    }
    return R;
}

bool rot_is_identity(const double *rot)
{
    if (rot == nullptr) return true;
    for (int a = 0; a < 9; ++a)
        if (rot[a] != ((a % 4) == 0 ? 1.0 : 0.0)) return false;
    return true;
}

// Workspace of the coherent direct path for one rotation.
struct DirectLayout {
    size_t points, partial, total;
};

DirectLayout direct_layout(const numag_sample *s, const Detector &d)
{
    DirectLayout L{};
    L.points = align_up((size_t)std::max<int64_t>(s->n_points, 1) * sizeof(PointRec));
    // partial sums of the full detector or of its Hermitian half, whichever is larger
    Detector dh = d;
    if (d.kind == NUMAG_GRID_CARTESIAN) {
        dh.n0 = (d.n0 + 1) / 2;
        const DirectPlan p = plan_direct_cartesian(d, s->n_points), ph = plan_direct_cartesian(dh, s->n_points);
        L.partial = std::max(p.nsplit > 1 ? align_up(direct_partial_bytes(p, d)) : 0,
                             ph.nsplit > 1 ? align_up(direct_partial_bytes(ph, dh)) : 0);
    } else {
        dh.n1 = std::max(1, d.n1 / 2);
        const DirectPlan p = plan_direct_polar(d, s->n_points), ph = plan_direct_polar(dh, s->n_points);
        L.partial = std::max(align_up(direct_partial_bytes(p, d)), align_up(direct_partial_bytes(ph, dh)));
    }
    L.total = L.points + L.partial;
    return L;
}

// Direct sums of one rotation: prep + sum + combine into amp (P x 8 doubles).  hermitian: evaluate half of the (centro-
// symmetric) detector and complete it by S(-q) = conj S(q) (real weights).
int run_direct(const numag_sample *s, const Rot &R, const Detector &d, double *amp, void *ws,
               hipStream_t st, bool hermitian = false)
{
    DirectLayout L = direct_layout(s, d);
    Carve cv(ws);
    PointRec *pts = (PointRec *)cv.take(L.points);
    double *part = (double *)cv.take(L.partial);
    const int64_t P = (int64_t)d.n0 * d.n1;
    if (s->n_points == 0 || (s->nuc == nullptr && s->mag == nullptr)) {
        return launch_fill(amp, P * 8, 0.0, st);
    }
    // channels summed: a sample without nuclear (magnetic) weights skips those FMAs
    const int channels = s->nuc == nullptr ? 3 : (s->mag == nullptr ? 1 : 4);
    int rc = launch_prepare_points(s->pos, s->nuc, s->mag, 0, s->n_points, s->regular, s->obj_offsets,
                                   s->n_objects, s->obj_pos, R, pts, st);
    if (rc != NUMAG_OK) return rc;
    if (d.kind == NUMAG_GRID_CARTESIAN) {
        Detector dh = d;
        if (hermitian) dh.n0 = (d.n0 + 1) / 2;  // rows [0, h): the first h n1 pixels of the output
        const int64_t Ph = (int64_t)dh.n0 * d.n1;
        DirectPlan p = plan_direct_cartesian(dh, s->n_points);
        p.channels = channels;
        if (p.nsplit == 1) {
            rc = launch_direct_cartesian(pts, s->n_points, dh, p, amp, st);
        } else {
            rc = launch_direct_cartesian(pts, s->n_points, dh, p, part, st);
            if (rc == NUMAG_OK) rc = launch_combine(part, p.nsplit, Ph, amp, 0, st);
        }
        if (rc != NUMAG_OK || !hermitian) return rc;
        return launch_mirror_cartesian(amp, P, Ph, st);
    }
    if (hermitian) {
        Detector dh = d;
        dh.n1 = d.n1 / 2;  // columns [0, n_theta / 2); their mirrors are m + n_theta / 2
        DirectPlan p = plan_direct_polar(dh, s->n_points);
        p.channels = channels;
        rc = launch_direct_polar(pts, s->n_points, dh, p, part, st);
        if (rc != NUMAG_OK) return rc;
        return launch_combine_polar_half(part, p.nsplit, d.n0, dh.n1, amp, st);
    }
    DirectPlan p = plan_direct_polar(d, s->n_points);
    p.channels = channels;
    rc = launch_direct_polar(pts, s->n_points, d, p, part, st);
    if (rc != NUMAG_OK) return rc;
    return launch_combine(part, p.nsplit, P, amp, 0, st);
}

unsigned long long next_plan_tag()
{
    static std::atomic<unsigned long long> counter{0};
    static const unsigned long long salt = [] {
        std::random_device rd;
        return ((unsigned long long)rd() << 32) ^ (unsigned long long)rd();
    }();
    // splitmix64 of (salt + counter): distinct for distinct counters, never reused in a process
    unsigned long long z = salt + 0x9E3779B97F4A7C15ull * (counter.fetch_add(1) + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Object-mode plan of a validated request.  rot may be NULL with n_rot == 1
// (identity); with rot NULL and n_rot > 1 only the sizes are meaningful.
std::unique_ptr<ObjPlan> make_plan(const numag_sample *s, int64_t n_rot, const double *rot, const Detector &d,
                                   int32_t path, int32_t mode, int32_t spec_per_object)
{
    auto pl = std::make_unique<ObjPlan>();
    pl->tag = next_plan_tag();
    pl->d = d;
    pl->path = path;
    pl->mode = mode;
    pl->spec_per_object = spec_per_object ? 1 : 0;
    pl->n_rot = n_rot;
    pl->K = s->n_objects;
    pl->W = s->n_points;
    pl->off.resize(s->n_objects + 1);
    if (s->n_objects == 1 || s->obj_offsets == nullptr) {
        pl->off[0] = 0;
        pl->off[1] = s->n_points;
    } else {
        std::memcpy(pl->off.data(), s->obj_offsets, sizeof(int64_t) * (s->n_objects + 1));
    }
    build_objects_plan(*pl);
    double *R = (double *)(pl->image.data() + pl->o_rot);
    if (rot != nullptr) {
        std::memcpy(R, rot, sizeof(double) * 9 * n_rot);
    } else {
        for (int a = 0; a < 9; ++a) R[a] = (a % 4) == 0 ? 1.0 : 0.0;
    }
    return pl;
}

int run_plan(const ObjPlan &pl, const numag_sample *s, double *amp_out, double *spec_out, void *ws, hipStream_t st)
{
    return launch_objects_plan(pl, *s, spec_out, amp_out, ws, st);
}

int upload_plan(const ObjPlan &pl, void *ws, hipStream_t st)
{
    NUMAG_HIP_CHECK(hipMemcpyAsync(ws, pl.image.data(), pl.image.size(), hipMemcpyHostToDevice, st));
    return NUMAG_OK;
}

size_t amplitudes_ws(const numag_sample *s, int64_t n_rot, const Detector &d, int32_t path, int32_t mode,
                     int32_t spec_per_object)
{
    if (is_separable(path))
        return align_up(separable_workspace_bytes(*s->regular, d, path, 1));
    if (mode == NUMAG_MODE_COHERENT) return direct_layout(s, d).total;
    return align_up(make_plan(s, n_rot, nullptr, d, path, mode, spec_per_object)->ws_bytes);
}

// Validation shared by numag_amplitudes and numag_plan_create.
int check_amplitudes_request(const numag_sample *sample, int64_t n_rot, const double *rot, const numag_qgrid *grid,
                             int32_t path, int32_t mode, const char *fn)
{
    int rc;
    if ((rc = check_sample(sample, fn)) != NUMAG_OK) return rc;
    if ((rc = check_grid(grid, fn)) != NUMAG_OK) return rc;
    if ((rc = check_rotations(rot, n_rot, fn)) != NUMAG_OK) return rc;
    const std::string f(fn);
    if (mode < NUMAG_MODE_COHERENT || mode > NUMAG_MODE_SPLIT) return invalid(f + ": unknown mode");
    if (path < NUMAG_PATH_DIRECT || path > NUMAG_PATH_SEPARABLE_F64_HERMITIAN) return invalid(f + ": unknown path");
    if (path == NUMAG_PATH_DIRECT_HERMITIAN && grid->kind == NUMAG_GRID_POLAR && grid->n1 % 2 != 0)
        return invalid(f + ": the Hermitian path needs an even n_theta on a polar detector");
    if (is_separable(path)) {
        if (sample->regular == nullptr) return invalid(f + ": separable path needs sample->regular");
        if (!rot_is_identity(rot) || n_rot != 1) return invalid(f + ": separable path needs the identity rotation");
        if (sample->n_objects != 1) return invalid(f + ": separable path needs one object");
        if (grid->kind != NUMAG_GRID_CARTESIAN) return invalid(f + ": separable path needs a Cartesian detector");
        if (mode != NUMAG_MODE_COHERENT) return invalid(f + ": separable path is COHERENT only");
    }
    if (mode != NUMAG_MODE_COHERENT) {
        if (mode == NUMAG_MODE_SPLIT && n_rot != 1) return invalid(f + ": SPLIT mode takes one rotation");
        if (sample->n_points > 0 && sample->pos == nullptr) {
            set_error(f + ": DILUTE/SPLIT modes need explicit positions");
            return NUMAG_E_UNSUPPORTED;
        }
        if (n_rot > (int64_t)1 << 30) return invalid(f + ": too many rotations");
    }
    return NUMAG_OK;
}

void delete_plan_cb(void *p) { delete (ObjPlan *)p; }

// The detector part a kernel evaluates on `path`: the whole detector, or the half
// of the Hermitian path (Cartesian rows [0, ceil(n0 / 2)), polar columns
// [0, n_theta / 2)).
Detector evaluated_detector(const Detector &d, int32_t path)
{
    Detector dh = d;
    if (path == NUMAG_PATH_DIRECT_HERMITIAN) {
        if (d.kind == NUMAG_GRID_CARTESIAN) dh.n0 = (d.n0 + 1) / 2;
        else dh.n1 = d.n1 / 2;
    }
    return dh;
}

// Device buffers the tuner allocates for its trial runs (freed on scope exit).
struct DeviceBuffers {
    std::vector<void *> bufs;
    ~DeviceBuffers()
    {
        for (void *b : bufs) (void)hipFree(b);
    }
    void *get(size_t bytes)
    {
        void *p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) return nullptr;
        bufs.push_back(p);
        return p;
    }
};

// Shortest time (ms) of `reps` runs of f() on st after one untimed run; < 0 on error.
template <class F>
double time_runs(F &&f, hipStream_t st, int reps)
{
    if (f() != NUMAG_OK) return -1.0;
    std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) e = nullptr;
    double best = -1.0;
    bool ok = true;
    for (int r = 0; r < reps && ok; ++r) {
        ok = ev[2 * r] != nullptr && ev[2 * r + 1] != nullptr && hipEventRecord(ev[2 * r], st) == hipSuccess &&
             f() == NUMAG_OK && hipEventRecord(ev[2 * r + 1], st) == hipSuccess;
    }
    if (ok && hipStreamSynchronize(st) == hipSuccess) {
        for (int r = 0; r < reps; ++r) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]) != hipSuccess) {
                best = -1.0;
                break;
            }
            if (best < 0.0 || ms < best) best = ms;
        }
    }
    for (auto &e : ev)
        if (e != nullptr) (void)hipEventDestroy(e);
    return best;
}

// Candidate shapes of a kernel on the evaluated detector d.
std::vector<TuneShape> tune_candidates(int kernel, const Detector &d, int64_t W)
{
    std::vector<TuneShape> c;
    const TuneShape def = default_tune_shape(kernel, d, W);
    if (kernel == kTuneDirect && d.kind == NUMAG_GRID_POLAR) {
        const std::vector<int> shapes = d.n0 <= 32 ? std::vector<int>{1, 0} : std::vector<int>{0, 2, 3, 4};
        for (int sh : shapes)
            for (int t : {256, 512, 1024}) c.push_back(TuneShape{sh, t * 8 / polar_shape_waves(sh)});
    } else if (kernel == kTuneObjects && d.kind == NUMAG_GRID_POLAR) {
        const std::vector<int> shapes = d.n0 <= 32 ? std::vector<int>{1, 0} : std::vector<int>{0, 2, 4};
        for (int sh : shapes)
            for (int t : {512, 1024, 2048}) c.push_back(TuneShape{sh, t});
    } else if (kernel == kTuneDirect || kernel == kTuneObjects) {
        const int l0 = def.shape;
        std::vector<int> lanes{l0};
        if (l0 > 8) lanes.push_back(l0 / 2);
        if (l0 < 64) lanes.push_back(l0 * 2);
        const std::vector<int> targets = kernel == kTuneDirect ? std::vector<int>{1024, 2048, 3072, 4096}
                                                               : std::vector<int>{1024, 2048, 4096};
        for (int l : lanes)
            for (int t : targets) c.push_back(TuneShape{l, t});
    } else {
        for (int t : {2048, 4096, 8192}) c.push_back(TuneShape{0, t});
    }
    // the default first (it is kept unless another shape is clearly faster)
    std::vector<TuneShape> out{def};
    for (const TuneShape &s : c)
        if (s.shape != def.shape || s.target != def.target) out.push_back(s);
    return out;
}

}  // namespace

int numag::validate_amplitudes_request(const numag_sample *sample, int64_t n_rot, const double *rot,
                                       const numag_qgrid *grid, int32_t path, int32_t mode, const char *fn)
{
    return check_amplitudes_request(sample, n_rot, rot, grid, path, mode, fn);
}

// The opaque plan handle of the C ABI.
struct numag_plan {
    std::unique_ptr<ObjPlan> p;
};

extern "C" {

size_t numag_correlation_2d_workspace_size(const numag_qgrid *grid, const numag_qgrid *rgrid)
{
    clear_error();
    if (check_grid(grid, "numag_correlation_2d_workspace_size") != NUMAG_OK) return 0;
    if (check_grid(rgrid, "numag_correlation_2d_workspace_size") != NUMAG_OK) return 0;
    return correlation_2d_workspace_bytes(make_detector(*grid), make_detector(*rgrid));
}

int numag_correlation_2d(const numag_qgrid *grid, const double *f, int32_t n_f, const numag_qgrid *rgrid,
                         double *C_out, void *workspace, size_t ws_bytes, void *stream)
{
    clear_error();
    int rc;
    if ((rc = check_grid(grid, "numag_correlation_2d")) != NUMAG_OK) return rc;
    if ((rc = check_grid(rgrid, "numag_correlation_2d")) != NUMAG_OK) return rc;
    if (n_f < 0) return invalid("numag_correlation_2d: n_f < 0");
    if (n_f > 0 && (f == nullptr || C_out == nullptr)) return invalid("numag_correlation_2d: NULL data or output");
    const Detector d = make_detector(*grid), rd = make_detector(*rgrid);
    const size_t need = correlation_2d_workspace_bytes(d, rd);
    if (ws_bytes < need || workspace == nullptr) {
        set_error("numag_correlation_2d: workspace too small (need " + std::to_string(need) + " bytes)");
        return NUMAG_E_WORKSPACE;
    }
    if (n_f == 0) return NUMAG_OK;
    return launch_correlation_2d(d, f, n_f, rd, C_out, workspace, ws_bytes, (hipStream_t)stream);
}

int numag_angular_spectrum(const numag_qgrid *grid, const double *f, int32_t n_f, int32_t k_max, double *Is_out,
                           double *Ic_out, double *As_out, double *Ac_out, void *stream)
{
    clear_error();
    int rc;
    if ((rc = check_grid(grid, "numag_angular_spectrum")) != NUMAG_OK) return rc;
    if (grid->kind != NUMAG_GRID_POLAR) return invalid("numag_angular_spectrum: needs a polar detector");
    if (n_f < 0 || k_max < 0) return invalid("numag_angular_spectrum: n_f and k_max must be >= 0");
    if (n_f > 65535) return invalid("numag_angular_spectrum: too many data sets");
    if (n_f > 0 && (f == nullptr || Is_out == nullptr || Ic_out == nullptr))
        return invalid("numag_angular_spectrum: NULL data or output");
    if ((As_out == nullptr) != (Ac_out == nullptr))
        return invalid("numag_angular_spectrum: give both or none of As_out, Ac_out");
    return launch_angular_spectrum(make_detector(*grid), f, n_f, k_max, Is_out, Ic_out, As_out, Ac_out,
                                   (hipStream_t)stream);
}

const char *numag_last_error(void) { return g_error.c_str(); }

const char *numag_version(void) { return "numag 0.1 (gfx950)"; }

size_t numag_workspace_size(const numag_sample *sample, int64_t n_rot, const numag_qgrid *grid,
                            int32_t path, int32_t mode)
{
    clear_error();
    if (check_sample(sample, "numag_workspace_size") != NUMAG_OK) return 0;
    if (check_grid(grid, "numag_workspace_size") != NUMAG_OK) return 0;
    if (mode < NUMAG_MODE_COHERENT || mode > NUMAG_MODE_SPLIT) {
        set_error("numag_workspace_size: unknown mode");
        return 0;
    }
    if (path < NUMAG_PATH_DIRECT || path > NUMAG_PATH_SEPARABLE_F64_HERMITIAN) {
        set_error("numag_workspace_size: unknown path");
        return 0;
    }
    if ((is_separable(path)) && sample->regular == nullptr) {
        set_error("numag_workspace_size: separable path needs a regular grid");
        return 0;
    }
    if (n_rot < 1) {
        set_error("numag_workspace_size: n_rot must be >= 1");
        return 0;
    }
    if (path == NUMAG_PATH_DIRECT_HERMITIAN && grid->kind == NUMAG_GRID_POLAR && grid->n1 % 2 != 0) {
        set_error("numag_workspace_size: the Hermitian path needs an even n_theta on a polar detector");
        return 0;
    }
    Detector d = make_detector(*grid);
    // object modes: enough for both spectral layouts (per object or summed)
    size_t amp = std::max(amplitudes_ws(sample, n_rot, d, path, mode, 0), amplitudes_ws(sample, n_rot, d, path, mode, 1));
    size_t grad = 0;
    if ((path == NUMAG_PATH_DIRECT || path == NUMAG_PATH_DIRECT_HERMITIAN) && mode == NUMAG_MODE_COHERENT) {
        // numag_grad: points + amplitudes (when not given) + direct partials + adjoint scratch
        const int64_t P = (int64_t)grid->n0 * grid->n1;
        grad = direct_layout(sample, d).total + align_up((size_t)P * 8 * sizeof(double)) +
               align_up(grad_workspace_bytes(d, sample->n_points, path == NUMAG_PATH_DIRECT_HERMITIAN));
    }
    return std::max(amp, grad);
}

int numag_amplitudes(const numag_sample *sample, int64_t n_rot, const double *rot, const numag_qgrid *grid,
                     int32_t path, int32_t mode, int32_t spec_per_object, double *amp_out, double *spec_out,
                     void *workspace, size_t ws_bytes, void *stream)
{
    clear_error();
    int rc;
    if ((rc = check_amplitudes_request(sample, n_rot, rot, grid, path, mode, "numag_amplitudes")) != NUMAG_OK)
        return rc;
    if ((mode == NUMAG_MODE_COHERENT || mode == NUMAG_MODE_SPLIT) && amp_out == nullptr)
        return invalid("numag_amplitudes: amp_out required in COHERENT/SPLIT mode");
    if ((mode == NUMAG_MODE_DILUTE || mode == NUMAG_MODE_SPLIT) && spec_out == nullptr)
        return invalid("numag_amplitudes: spec_out required in DILUTE/SPLIT mode");
    Detector d = make_detector(*grid);
    hipStream_t st = (hipStream_t)stream;
    const int64_t P = (int64_t)grid->n0 * grid->n1;
    if (mode != NUMAG_MODE_COHERENT) {
        // a one-off plan: its image is uploaded here and freed once the stream has copied it
        std::unique_ptr<ObjPlan> pl = make_plan(sample, n_rot, rot, d, path, mode, spec_per_object);
        const size_t need = align_up(pl->ws_bytes);
        if (ws_bytes < need || workspace == nullptr) {
            set_error("numag_amplitudes: workspace too small (need " + std::to_string(need) + " bytes)");
            return NUMAG_E_WORKSPACE;
        }
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        NUMAG_HIP_CHECK(hipStreamIsCapturing(st, &cap));
        if (cap != hipStreamCaptureStatusNone) {
            set_error("numag_amplitudes: DILUTE/SPLIT modes upload their tables on every call; under graph capture "
                      "create a plan (numag_plan_create), upload it once and capture numag_amplitudes_plan");
            return NUMAG_E_UNSUPPORTED;
        }
        rc = upload_plan(*pl, workspace, st);
        if (rc == NUMAG_OK)
            rc = run_plan(*pl, sample, mode == NUMAG_MODE_SPLIT ? amp_out : nullptr, spec_out, workspace, st);
        if (rc == NUMAG_OK && hipLaunchHostFunc(st, delete_plan_cb, pl.get()) == hipSuccess) {
            pl.release();  // deleted by the stream callback
            return NUMAG_OK;
        }
        (void)hipStreamSynchronize(st);  // error path: the copy may still read the image
        return rc != NUMAG_OK ? rc : NUMAG_E_HIP;
    }
    const size_t need = amplitudes_ws(sample, n_rot, d, path, mode, 0);
    if (ws_bytes < need || (need > 0 && workspace == nullptr)) {
        set_error("numag_amplitudes: workspace too small (need " + std::to_string(need) + " bytes)");
        return NUMAG_E_WORKSPACE;
    }
    if (is_separable(path))
        return launch_separable(sample->nuc, sample->mag, *sample->regular, d, path, 1, amp_out, workspace,
                                ws_bytes, st);
    for (int64_t r = 0; r < n_rot; ++r) {
        rc = run_direct(sample, rot_of(rot, r), d, amp_out + r * P * 8, workspace, st,
                        path == NUMAG_PATH_DIRECT_HERMITIAN);
        if (rc != NUMAG_OK) return rc;
    }
    return NUMAG_OK;
}

int numag_plan_create(const numag_sample *sample, int64_t n_rot, const double *rot, const numag_qgrid *grid,
                      int32_t path, int32_t mode, int32_t spec_per_object, numag_plan **plan_out)
{
    clear_error();
    if (plan_out == nullptr) return invalid("numag_plan_create: plan_out is NULL");
    *plan_out = nullptr;
    int rc;
    if ((rc = check_amplitudes_request(sample, n_rot, rot, grid, path, mode, "numag_plan_create")) != NUMAG_OK)
        return rc;
    if (mode != NUMAG_MODE_DILUTE && mode != NUMAG_MODE_SPLIT)
        return invalid("numag_plan_create: plans are for DILUTE and SPLIT modes");
    if (path != NUMAG_PATH_DIRECT && path != NUMAG_PATH_DIRECT_HERMITIAN)
        return invalid("numag_plan_create: path must be NUMAG_PATH_DIRECT or NUMAG_PATH_DIRECT_HERMITIAN");
    auto h = std::make_unique<numag_plan>();
    h->p = make_plan(sample, n_rot, rot, make_detector(*grid), path, mode, spec_per_object);
    *plan_out = h.release();
    return NUMAG_OK;
}

size_t numag_plan_workspace_size(const numag_plan *plan)
{
    clear_error();
    if (plan == nullptr) {
        set_error("numag_plan_workspace_size: plan is NULL");
        return 0;
    }
    return align_up(plan->p->ws_bytes);
}

int numag_plan_upload(const numag_plan *plan, void *workspace, size_t ws_bytes, void *stream)
{
    clear_error();
    if (plan == nullptr) return invalid("numag_plan_upload: plan is NULL");
    if (workspace == nullptr || ws_bytes < align_up(plan->p->ws_bytes)) {
        set_error("numag_plan_upload: workspace too small (need " + std::to_string(align_up(plan->p->ws_bytes)) +
                  " bytes)");
        return NUMAG_E_WORKSPACE;
    }
    return upload_plan(*plan->p, workspace, (hipStream_t)stream);
}

int numag_amplitudes_plan(const numag_plan *plan, const numag_sample *sample, double *amp_out, double *spec_out,
                          void *workspace, size_t ws_bytes, void *stream)
{
    clear_error();
    int rc;
    if (plan == nullptr) return invalid("numag_amplitudes_plan: plan is NULL");
    const ObjPlan &pl = *plan->p;
    if ((rc = check_sample(sample, "numag_amplitudes_plan")) != NUMAG_OK) return rc;
    if (sample->n_points != pl.W || sample->n_objects != pl.K)
        return invalid("numag_amplitudes_plan: the sample's point or object count differs from the plan's");
    if (pl.K > 1 && std::memcmp(sample->obj_offsets, pl.off.data(), sizeof(int64_t) * (pl.K + 1)) != 0)
        return invalid("numag_amplitudes_plan: the sample's object offsets differ from the plan's");
    if (sample->n_points > 0 && sample->pos == nullptr) {
        set_error("numag_amplitudes_plan: DILUTE/SPLIT modes need explicit positions");
        return NUMAG_E_UNSUPPORTED;
    }
    if (pl.mode == NUMAG_MODE_SPLIT && amp_out == nullptr)
        return invalid("numag_amplitudes_plan: amp_out required in SPLIT mode");
    if (spec_out == nullptr) return invalid("numag_amplitudes_plan: spec_out is NULL");
    if (workspace == nullptr || ws_bytes < align_up(pl.ws_bytes)) {
        set_error("numag_amplitudes_plan: workspace too small (need " + std::to_string(align_up(pl.ws_bytes)) +
                  " bytes)");
        return NUMAG_E_WORKSPACE;
    }
    return run_plan(pl, sample, pl.mode == NUMAG_MODE_SPLIT ? amp_out : nullptr, spec_out, workspace,
                    (hipStream_t)stream);
}

void numag_plan_destroy(numag_plan *plan) { delete plan; }

static int check_snapshots(const numag_regular *points, int64_t n_snap, const numag_qgrid *grid, int32_t path,
                           const char *fn)
{
    int rc;
    if (points == nullptr) return invalid(std::string(fn) + ": points is NULL");
    if (n_snap < 1) return invalid(std::string(fn) + ": n_snap must be >= 1");
    if ((rc = check_grid(grid, fn)) != NUMAG_OK) return rc;
    if (!is_separable(path))
        return invalid(std::string(fn) + ": snapshots run on the separable paths");
    if (grid->kind != NUMAG_GRID_CARTESIAN) return invalid(std::string(fn) + ": separable path needs a Cartesian detector");
    numag_sample smp{};
    smp.n_points = (int64_t)points->n[0] * points->n[1] * points->n[2];
    smp.n_objects = 1;
    smp.regular = points;
    if ((rc = check_sample(&smp, fn)) != NUMAG_OK) return rc;
    // 4 n_snap channel sets index the contraction tiles as int
    const int64_t tiles = 4 * n_snap * (((int64_t)grid->n0 + 15) / 16) * (((int64_t)grid->n1 + 15) / 16);
    if (tiles > ((int64_t)1 << 31) - 4) return invalid(std::string(fn) + ": too many snapshots for one call");
    return NUMAG_OK;
}

size_t numag_snapshots_workspace_size(const numag_regular *points, int64_t n_snap, const numag_qgrid *grid,
                                      int32_t path)
{
    clear_error();
    if (check_snapshots(points, n_snap, grid, path, "numag_snapshots_workspace_size") != NUMAG_OK) return 0;
    return align_up(separable_workspace_bytes(*points, make_detector(*grid), path, n_snap));
}

int numag_amplitudes_snapshots(const numag_regular *points, int64_t n_snap, const double *nuc, const double *mag,
                               const numag_qgrid *grid, int32_t path, double *amp_out, void *workspace,
                               size_t ws_bytes, void *stream)
{
    clear_error();
    int rc;
    if ((rc = check_snapshots(points, n_snap, grid, path, "numag_amplitudes_snapshots")) != NUMAG_OK) return rc;
    if (amp_out == nullptr) return invalid("numag_amplitudes_snapshots: amp_out is NULL");
    const Detector d = make_detector(*grid);
    const size_t need = align_up(separable_workspace_bytes(*points, d, path, n_snap));
    if (ws_bytes < need || workspace == nullptr) {
        set_error("numag_amplitudes_snapshots: workspace too small (need " + std::to_string(need) + " bytes)");
        return NUMAG_E_WORKSPACE;
    }
    return launch_separable(nuc, mag, *points, d, path, n_snap, amp_out, workspace, ws_bytes, (hipStream_t)stream);
}

int numag_spectral_matrix(const numag_qgrid *grid, int64_t n_sets, const double *amp, double *spec_out,
                          void *stream)
{
    clear_error();
    int rc;
    if ((rc = check_grid(grid, "numag_spectral_matrix")) != NUMAG_OK) return rc;
    if (n_sets < 0) return invalid("numag_spectral_matrix: n_sets < 0");
    if (n_sets > 0 && (amp == nullptr || spec_out == nullptr))
        return invalid("numag_spectral_matrix: amp and spec_out are required");
    return launch_spectral_matrix(n_sets, (int64_t)grid->n0 * grid->n1, amp, spec_out, (hipStream_t)stream);
}

int numag_cross_section(const numag_qgrid *grid, int64_t n_sets, const double *amp, const double *spec,
                        const numag_consts *consts, uint32_t obs_mask, double *out, void *stream)
{
    clear_error();
    int rc;
    if ((rc = check_grid(grid, "numag_cross_section")) != NUMAG_OK) return rc;
    if (n_sets < 0) return invalid("numag_cross_section: n_sets < 0");
    if (amp != nullptr && spec != nullptr) return invalid("numag_cross_section: give exactly one of amp and spec");
    if (n_sets > 0 && amp == nullptr && spec == nullptr)
        return invalid("numag_cross_section: give exactly one of amp and spec");
    if (consts == nullptr) return invalid("numag_cross_section: consts is NULL");
    if (!(consts->V > 0.0) || !is_finite(consts->V)) return invalid("numag_cross_section: V must be > 0");
    if (!is_finite(consts->bH) || !is_finite(consts->scale)) return invalid("numag_cross_section: bH/scale not finite");
    for (int a = 0; a < 3; ++a)
        if (!is_finite(consts->P[a])) return invalid("numag_cross_section: P not finite");
    if (obs_mask == 0 || (obs_mask & ~NUMAG_OBS_ALL) != 0)
        return invalid("numag_cross_section: obs_mask empty or has unknown bits");
    if (out == nullptr && n_sets > 0) return invalid("numag_cross_section: out is NULL");
    return launch_cross_section(make_detector(*grid), n_sets, amp, spec, *consts, obs_mask, out,
                                (hipStream_t)stream);
}

int numag_azimuthal_average(const numag_qgrid *grid, const double *f, int32_t n_f, int32_t n_bins,
                            double qmax_avg, double *I_out, int64_t *count_out, void *stream)
{
    clear_error();
    int rc;
    if ((rc = check_grid(grid, "numag_azimuthal_average")) != NUMAG_OK) return rc;
    if (n_f < 0 || n_bins < 1) return invalid("numag_azimuthal_average: need n_f >= 0 and n_bins >= 1");
    if (n_f > 65535 || n_bins > (1 << 24)) return invalid("numag_azimuthal_average: n_f or n_bins too large");
    if (f == nullptr && n_f > 0) return invalid("numag_azimuthal_average: f is NULL");
    if (I_out == nullptr && n_f > 0) return invalid("numag_azimuthal_average: I_out is NULL");
    if (grid->kind == NUMAG_GRID_POLAR) {
        if (n_bins != grid->n0) return invalid("numag_azimuthal_average: polar detector needs n_bins == n_q");
    } else if (!(qmax_avg > 0.0) || !is_finite(qmax_avg)) {
        return invalid("numag_azimuthal_average: qmax_avg must be > 0");
    }
    return launch_azimuthal(make_detector(*grid), f, n_f, n_bins, qmax_avg, I_out, count_out,
                            (hipStream_t)stream);
}

int numag_correlation(const double *q, const double *I, int32_t n_q, int32_t n_f, const double *r, int32_t n_r,
                      double scale, double *c_out, double *p_out, void *stream)
{
    clear_error();
    if (n_q < 0 || n_f < 0 || n_r < 0) return invalid("numag_correlation: negative size");
    if ((n_q > 0 && (q == nullptr || (n_f > 0 && I == nullptr))) || (n_r > 0 && r == nullptr))
        return invalid("numag_correlation: NULL input");
    if ((int64_t)n_f * n_r > 0 && (c_out == nullptr || p_out == nullptr))
        return invalid("numag_correlation: NULL output");
    if (!is_finite(scale)) return invalid("numag_correlation: scale not finite");
    return launch_correlation(q, I, n_q, n_f, r, n_r, scale, c_out, p_out, (hipStream_t)stream);
}

int numag_grad(const numag_sample *sample, const double *rot, const numag_qgrid *grid,
               const numag_consts *consts, const double *amp_in, const double *target, const double *weight,
               double *loss_out, double *dnuc_out, double *dmag_out, void *workspace, size_t ws_bytes,
               void *stream)
{
    return numag_grad_path(sample, rot, grid, NUMAG_PATH_DIRECT, consts, amp_in, target, weight, loss_out, dnuc_out,
                           dmag_out, workspace, ws_bytes, stream);
}

int numag_grad_path(const numag_sample *sample, const double *rot, const numag_qgrid *grid, int32_t path,
                    const numag_consts *consts, const double *amp_in, const double *target, const double *weight,
                    double *loss_out, double *dnuc_out, double *dmag_out, void *workspace, size_t ws_bytes,
                    void *stream)
{
    clear_error();
    int rc;
    if (path != NUMAG_PATH_DIRECT && path != NUMAG_PATH_DIRECT_HERMITIAN)
        return invalid("numag_grad: path must be NUMAG_PATH_DIRECT or NUMAG_PATH_DIRECT_HERMITIAN");
    const bool hermitian = path == NUMAG_PATH_DIRECT_HERMITIAN;
    if ((rc = check_sample(sample, "numag_grad")) != NUMAG_OK) return rc;
    if ((rc = check_grid(grid, "numag_grad")) != NUMAG_OK) return rc;
    if ((rc = check_rotations(rot, 1, "numag_grad")) != NUMAG_OK) return rc;
    if (consts == nullptr || !(consts->V > 0.0)) return invalid("numag_grad: consts missing or V <= 0");
    if (weight == nullptr) return invalid("numag_grad: weight is required");
    if (target != nullptr && loss_out == nullptr)
        return invalid("numag_grad: loss_out is required when a target is given");
    if (hermitian && grid->kind == NUMAG_GRID_POLAR && grid->n1 % 2 != 0)
        return invalid("numag_grad: the Hermitian path needs an even n_theta on a polar detector");
    Detector d = make_detector(*grid);
    const int64_t P = (int64_t)grid->n0 * grid->n1;
    DirectLayout L = direct_layout(sample, d);
    const size_t gbytes = grad_workspace_bytes(d, sample->n_points, hermitian);
    const size_t need = L.total + align_up((size_t)P * 8 * sizeof(double)) + align_up(gbytes);
    if (ws_bytes < need || workspace == nullptr) {
        set_error("numag_grad: workspace too small (need " + std::to_string(need) + " bytes)");
        return NUMAG_E_WORKSPACE;
    }
    hipStream_t st = (hipStream_t)stream;
    Carve cv(workspace);
    char *direct_ws = (char *)cv.take(L.total);
    double *amp = (double *)cv.take((size_t)P * 8 * sizeof(double));
    void *gws = cv.take(gbytes);
    const Rot R = rot_of(rot, 0);
    if (amp_in == nullptr) {
        rc = run_direct(sample, R, d, amp, direct_ws, st, hermitian);
        if (rc != NUMAG_OK) return rc;
        amp_in = amp;
    } else {
        // points only
        rc = launch_prepare_points(sample->pos, sample->nuc, sample->mag, 0, sample->n_points, sample->regular,
                                   sample->obj_offsets, sample->n_objects, sample->obj_pos, R,
                                   (PointRec *)direct_ws, st);
        if (rc != NUMAG_OK) return rc;
    }
    const PointRec *pts = (const PointRec *)direct_ws;
    return launch_grad(pts, sample->n_points, d, *consts, amp_in, target, weight, loss_out, dnuc_out, dmag_out,
                       R, gws, gbytes, st, hermitian);
}

int numag_tune_get(int32_t kernel, const numag_qgrid *grid, int32_t path, int64_t n_points,
                   numag_tune_shape *default_out, numag_tune_shape *current_out)
{
    clear_error();
    int rc;
    if ((rc = check_grid(grid, "numag_tune_get")) != NUMAG_OK) return rc;
    if (kernel < 0 || kernel >= kTuneKernelCount) return invalid("numag_tune_get: unknown kernel");
    if (path != NUMAG_PATH_DIRECT && path != NUMAG_PATH_DIRECT_HERMITIAN)
        return invalid("numag_tune_get: path must be NUMAG_PATH_DIRECT or NUMAG_PATH_DIRECT_HERMITIAN");
    if (n_points < 0) return invalid("numag_tune_get: n_points < 0");
    const Detector d = evaluated_detector(make_detector(*grid), path);
    const TuneShape def = default_tune_shape(kernel, d, n_points), cur = current_tune_shape(kernel, d, n_points);
    if (default_out != nullptr) *default_out = numag_tune_shape{def.shape, def.target};
    if (current_out != nullptr) *current_out = numag_tune_shape{cur.shape, cur.target};
    TuneShape t{};
    return tuned_shape(kernel, d, n_points, &t) && valid_tune_shape(kernel, d, t) ? 1 : 0;
}

int numag_tune_set(int32_t kernel, const numag_qgrid *grid, int32_t path, int64_t n_points,
                   const numag_tune_shape *shape)
{
    clear_error();
    int rc;
    if ((rc = check_grid(grid, "numag_tune_set")) != NUMAG_OK) return rc;
    if (kernel < 0 || kernel >= kTuneKernelCount) return invalid("numag_tune_set: unknown kernel");
    if (path != NUMAG_PATH_DIRECT && path != NUMAG_PATH_DIRECT_HERMITIAN)
        return invalid("numag_tune_set: path must be NUMAG_PATH_DIRECT or NUMAG_PATH_DIRECT_HERMITIAN");
    if (n_points < 0) return invalid("numag_tune_set: n_points < 0");
    const Detector d = evaluated_detector(make_detector(*grid), path);
    if (shape == nullptr) {
        tune_erase(kernel, d, n_points);
        return NUMAG_OK;
    }
    const TuneShape s{shape->shape, shape->target};
    if (!valid_tune_shape(kernel, d, s)) return invalid("numag_tune_set: shape not valid for this kernel and detector");
    tune_store(kernel, d, n_points, s, 0.0, 0.0);
    return NUMAG_OK;
}

int numag_tune_clear(void)
{
    clear_error();
    tune_clear();
    return NUMAG_OK;
}

int numag_autotune(const numag_sample *sample, int64_t n_rot, const double *rot, const numag_qgrid *grid,
                   int32_t path, int32_t kernel, int64_t max_points, numag_tune_shape *chosen_out, void *stream)
{
    clear_error();
    int rc;
    const char *fn = "numag_autotune";
    if (kernel < 0 || kernel >= kTuneKernelCount) return invalid("numag_autotune: unknown kernel");
    if (path != NUMAG_PATH_DIRECT && path != NUMAG_PATH_DIRECT_HERMITIAN)
        return invalid("numag_autotune: path must be NUMAG_PATH_DIRECT or NUMAG_PATH_DIRECT_HERMITIAN");
    const int32_t mode = kernel == kTuneObjects ? NUMAG_MODE_DILUTE : NUMAG_MODE_COHERENT;
    if ((rc = check_amplitudes_request(sample, n_rot, rot, grid, path, mode, fn)) != NUMAG_OK) return rc;
    if (max_points < 0) return invalid("numag_autotune: max_points < 0");
    hipStream_t st = (hipStream_t)stream;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    NUMAG_HIP_CHECK(hipStreamIsCapturing(st, &cap));
    if (cap != hipStreamCaptureStatusNone) {
        set_error("numag_autotune: waits for the stream and allocates; not under graph capture");
        return NUMAG_E_UNSUPPORTED;
    }
    const Detector dfull = make_detector(*grid);
    const Detector d = kernel == kTuneObjects ? objects_detector(dfull, path == NUMAG_PATH_DIRECT_HERMITIAN)
                                              : evaluated_detector(dfull, path);
    const int64_t W = sample->n_points;
    const int64_t P = (int64_t)grid->n0 * grid->n1;
    // the trial sample: coherent kernels time the first max_points points as one
    // object (object offsets move points, they do not change the work)
    numag_sample ts = *sample;
    if (kernel != kTuneObjects) {
        ts.n_objects = 1;
        ts.obj_offsets = nullptr;
        ts.obj_pos = nullptr;
        if (max_points > 0 && max_points < W && ts.regular == nullptr) ts.n_points = max_points;
    }
    const int64_t n_rot_t = kernel == kTuneObjects ? std::min<int64_t>(n_rot, 64) : 1;
    const std::vector<TuneShape> cands = tune_candidates(kernel, d, W);
    // buffers: outputs, and a workspace large enough for every candidate
    DeviceBuffers mem;
    double *amp = (double *)mem.get((size_t)P * 8 * sizeof(double));
    double *spec = nullptr, *target = nullptr, *weight = nullptr, *loss = nullptr, *dn = nullptr, *dm = nullptr;
    if (kernel == kTuneObjects) spec = (double *)mem.get((size_t)P * 16 * sizeof(double) *
                                                         (size_t)std::max<int64_t>(1, sample->n_objects));
    if (kernel == kTuneAdjoint) {
        target = (double *)mem.get((size_t)P * sizeof(double));
        weight = (double *)mem.get((size_t)P * sizeof(double));
        loss = (double *)mem.get(sizeof(double));
        dn = (double *)mem.get((size_t)ts.n_points * sizeof(double));
        dm = (double *)mem.get((size_t)ts.n_points * 3 * sizeof(double));
        if (target == nullptr || weight == nullptr || loss == nullptr || dn == nullptr || dm == nullptr) {
            set_error("numag_autotune: hipMalloc failed");
            return NUMAG_E_HIP;
        }
        if ((rc = launch_fill(target, P, 0.0, st)) != NUMAG_OK) return rc;
        if ((rc = launch_fill(weight, P, 1.0, st)) != NUMAG_OK) return rc;
    }
    if (amp == nullptr || (kernel == kTuneObjects && spec == nullptr)) {
        set_error("numag_autotune: hipMalloc failed");
        return NUMAG_E_HIP;
    }
    // trial runs read their shape from the table under the trial point count Wt;
    // the result is stored under the sample's W.  An entry already held under Wt
    // is put back afterwards (or if tuning fails).
    const int64_t Wt = ts.n_points;
    TuneShape prev{};
    const bool had_prev = tuned_shape(kernel, d, Wt, &prev);
    auto restore = [&]() {
        if (had_prev) tune_store(kernel, d, Wt, prev, 0.0, 0.0);
        else tune_erase(kernel, d, Wt);
    };
    size_t ws_need = 0;
    for (const TuneShape &c : cands) {
        tune_store(kernel, d, Wt, c, 0.0, 0.0);
        size_t need = 0;
        if (kernel == kTuneObjects) {
            need = make_plan(sample, n_rot_t, nullptr, dfull, path, NUMAG_MODE_DILUTE, 1)->ws_bytes;
        } else {
            const Detector &dd = dfull;
            need = direct_layout(&ts, dd).total + align_up((size_t)P * 8 * sizeof(double)) +
                   align_up(grad_workspace_bytes(dd, ts.n_points, path == NUMAG_PATH_DIRECT_HERMITIAN));
        }
        ws_need = std::max(ws_need, align_up(need));
    }
    void *ws = mem.get(ws_need);
    if (ws == nullptr) {
        restore();
        set_error("numag_autotune: hipMalloc of the trial workspace failed");
        return NUMAG_E_HIP;
    }
    const bool herm = path == NUMAG_PATH_DIRECT_HERMITIAN;
    const Rot R = rot_of(rot, 0);
    if (kernel == kTuneAdjoint) {  // the sums the residual weights are formed from
        if ((rc = run_direct(&ts, R, dfull, amp, ws, st, herm)) != NUMAG_OK) {
            restore();
            return rc;
        }
    }
    double best_ms = -1.0, default_ms = -1.0;
    TuneShape best = cands[0];
    for (size_t i = 0; i < cands.size(); ++i) {
        const TuneShape &c = cands[i];
        tune_store(kernel, d, Wt, c, 0.0, 0.0);
        std::unique_ptr<ObjPlan> pl;
        if (kernel == kTuneObjects) {
            pl = make_plan(sample, n_rot_t, rot, dfull, path, NUMAG_MODE_DILUTE, 1);
            rc = upload_plan(*pl, ws, st);
            if (rc == NUMAG_OK && hipStreamSynchronize(st) != hipSuccess) rc = NUMAG_E_HIP;
            if (rc != NUMAG_OK) {
                restore();
                return rc;
            }
        }
        auto run = [&]() -> int {
            if (kernel == kTuneObjects) return run_plan(*pl, sample, nullptr, spec, ws, st);
            if (kernel == kTuneDirect) return run_direct(&ts, R, dfull, amp, ws, st, herm);
            const DirectLayout L = direct_layout(&ts, dfull);
            char *base = (char *)ws;
            const int r1 = launch_prepare_points(ts.pos, ts.nuc, ts.mag, 0, ts.n_points, ts.regular, nullptr, 1,
                                                 nullptr, R, (PointRec *)base, st);
            if (r1 != NUMAG_OK) return r1;
            numag_consts k{1.0, 1.0, 1.0, {0.0, 0.0, 1.0}};
            return launch_grad((const PointRec *)base, ts.n_points, dfull, k, amp, target, weight, loss, dn, dm, R,
                               base + L.total + align_up((size_t)P * 8 * sizeof(double)),
                               grad_workspace_bytes(dfull, ts.n_points, herm), st, herm);
        };
        // one trial run to size the repetitions: about 0.3 s of timed work per candidate
        double t1 = time_runs(run, st, 1);
        if (t1 < 0.0) {
            restore();
            if (numag_last_error()[0] == 0) set_error("numag_autotune: a trial run failed");
            return NUMAG_E_HIP;
        }
        if (i == 0) {
            // the engine clock settles after some tens of ms of load: run the first
            // candidate for about 40 ms before any candidate is timed
            const int warm = (int)std::min(200.0, std::ceil(40.0 / std::max(t1, 1e-3)));
            for (int w = 0; w < warm; ++w)
                if ((rc = run()) != NUMAG_OK) {
                    restore();
                    return rc;
                }
            t1 = time_runs(run, st, 1);
            if (t1 < 0.0) {
                restore();
                if (numag_last_error()[0] == 0) set_error("numag_autotune: a trial run failed");
                return NUMAG_E_HIP;
            }
        }
        const int reps = (int)std::max(1.0, std::min(5.0, 300.0 / std::max(t1, 1e-3)));
        const double t = reps > 1 ? std::min(t1, time_runs(run, st, reps)) : t1;
        if (i == 0) default_ms = t;
        if (best_ms < 0.0 || t < best_ms) {
            best_ms = t;
            best = c;
        }
    }
    // keep the default unless another shape is faster by more than 1 %
    if (best_ms > 0.99 * default_ms) {
        best = cands[0];
        best_ms = default_ms;
    }
    if (Wt != W) restore();
    tune_store(kernel, d, W, best, best_ms, default_ms);
    if (chosen_out != nullptr) *chosen_out = numag_tune_shape{best.shape, best.target};
    return tune_save();
}

}  // extern "C"
