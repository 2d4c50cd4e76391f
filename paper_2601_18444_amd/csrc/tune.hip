// Tile-shape autotuner of the sum kernels: a process-wide table of launch shapes
// keyed by (kernel, detector kind and evaluated size, point-count class, GPU
// architecture), filled by timing candidate shapes on the caller's own inputs
// (numag_autotune) or set directly (numag_tune_set), and optionally kept in a
// text file named by NUMAG_AUTOTUNE_CACHE (read on the first lookup, rewritten
// after every tuning run).  A shape only changes how work is cut into
// workgroups and point splits -- which pixels a lane owns, how many points a
// workgroup sums -- never what is summed: sums under different shapes agree to
// rounding.
//
// Shapes per kernel:
//   direct, Cartesian detector: lanes per detector row (8, 16, 32, 64) and the
//     workgroups a launch aims for (split over points);
//   direct, polar detector: one of the polar kernel's workgroup shapes
//     (64 x 64, 32 x 64, 128 x 32, 256 x 16 single- or double-buffered) and the
//     workgroups aimed for;
//   adjoint: the workgroups aimed for (point blocks x detector ranges);
//   objects (persistent kernel): lanes per detector row (polar: the workgroup
//     shape) and the work items aimed for.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "numag_internal.h"

namespace numag {
namespace {

struct Key {
    std::string arch;
    int kernel, kind, n0, n1, wclass;
    bool operator<(const Key &o) const
    {
        return std::tie(arch, kernel, kind, n0, n1, wclass) < std::tie(o.arch, o.kernel, o.kind, o.n0, o.n1, o.wclass);
    }
};

struct Entry {
    TuneShape shape;
    double ms, default_ms;  // measured by numag_autotune (0 when set directly or unknown)
};

std::mutex g_mu;
std::map<Key, Entry> g_table;
bool g_loaded = false;

const char *kKernelNames[kTuneKernelCount] = {"direct", "adjoint", "objects"};

const std::string &device_arch()
{
    static const std::string arch = [] {
        int dev = 0;
        hipDeviceProp_t prop{};
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return std::string("gfx950");
        std::string a = prop.gcnArchName;
        const size_t colon = a.find(':');
        return colon == std::string::npos ? a : a.substr(0, colon);
    }();
    return arch;
}

std::string cache_path()
{
    const char *e = getenv("NUMAG_AUTOTUNE_CACHE");
    return e != nullptr ? std::string(e) : std::string();
}

// One entry per line: arch kernel kind n0 n1 wclass shape target ms default_ms
void load_locked()
{
    if (g_loaded) return;
    g_loaded = true;
    const std::string path = cache_path();
    if (path.empty()) return;
    FILE *f = fopen(path.c_str(), "r");
    if (f == nullptr) return;
    char line[512];
    while (fgets(line, sizeof line, f) != nullptr) {
        if (line[0] == '#') continue;
        char arch[64], kname[32];
        int kind, n0, n1, wc, shape, target;
        double ms, dms;
        if (sscanf(line, "%63s %31s %d %d %d %d %d %d %lf %lf", arch, kname, &kind, &n0, &n1, &wc, &shape, &target,
                   &ms, &dms) != 10)
            continue;
        int kernel = -1;
        for (int k = 0; k < kTuneKernelCount; ++k)
            if (strcmp(kname, kKernelNames[k]) == 0) kernel = k;
        if (kernel < 0) continue;
        g_table[Key{arch, kernel, kind, n0, n1, wc}] = Entry{TuneShape{shape, target}, ms, dms};
    }
    fclose(f);
}

int save_locked()
{
    const std::string path = cache_path();
    if (path.empty()) return NUMAG_OK;
    const std::string tmp = path + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (f == nullptr) {
        set_error("numag_autotune: cannot write " + tmp);
        return NUMAG_E_INVALID;
    }
    fprintf(f, "# numag launch shapes: arch kernel kind n0 n1 wclass shape target ms default_ms\n");
    for (const auto &kv : g_table) {
        const Key &k = kv.first;
        const Entry &e = kv.second;
        fprintf(f, "%s %s %d %d %d %d %d %d %.6f %.6f\n", k.arch.c_str(), kKernelNames[k.kernel], k.kind, k.n0, k.n1,
                k.wclass, e.shape.shape, e.shape.target, e.ms, e.default_ms);
    }
    fclose(f);
    if (rename(tmp.c_str(), path.c_str()) != 0) {
        set_error("numag_autotune: cannot replace " + path);
        return NUMAG_E_INVALID;
    }
    return NUMAG_OK;
}

Key make_key(int kernel, const Detector &d, int64_t W)
{
    return Key{device_arch(), kernel, d.kind, d.n0, d.n1, tune_wclass(W)};
}

}  // namespace

int tune_wclass(int64_t W)
{
    if (W <= 1) return 0;
    return (int)std::floor(2.0 * std::log2((double)W));  // half-octaves
}

bool tuned_shape(int kernel, const Detector &d, int64_t W, TuneShape *out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    const auto it = g_table.find(make_key(kernel, d, W));
    if (it == g_table.end()) return false;
    *out = it->second.shape;
    return true;
}

void tune_store(int kernel, const Detector &d, int64_t W, const TuneShape &s, double ms, double default_ms)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    g_table[make_key(kernel, d, W)] = Entry{s, ms, default_ms};
}

void tune_erase(int kernel, const Detector &d, int64_t W)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    g_table.erase(make_key(kernel, d, W));
}

int tune_save()
{
    std::lock_guard<std::mutex> lk(g_mu);
    return save_locked();
}

void tune_clear()
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
    g_loaded = true;  // a cleared table is not reloaded from the cache file
}

bool valid_tune_shape(int kernel, const Detector &d, const TuneShape &s)
{
    if (s.target < 0 || s.target > (1 << 20)) return false;
    switch (kernel) {
        case kTuneDirect:
            if (d.kind == NUMAG_GRID_POLAR) return s.shape >= 0 && s.shape < kPolarShapeCount && (s.shape != 1 || d.n0 <= 32);
            return s.shape == 8 || s.shape == 16 || s.shape == 32 || s.shape == 64;
        case kTuneAdjoint:
            return s.shape == 0;
        case kTuneObjects:
            if (d.kind == NUMAG_GRID_POLAR) return s.shape >= 0 && s.shape < kPolarShapeCount && (s.shape != 1 || d.n0 <= 32);
            return s.shape == 8 || s.shape == 16 || s.shape == 32 || s.shape == 64;
        default:
            return false;
    }
}

}  // namespace numag
