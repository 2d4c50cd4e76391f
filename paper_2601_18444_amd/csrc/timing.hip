// Kernel timer behind numag_kernel_timer / numag_kernel_timer_read: HIP event
// pairs recorded on the launching stream around the sum kernels.
#include <mutex>
#include <vector>

#include "numag_internal.h"

namespace numag {

namespace {

struct Record {
    int id;
    int kernel;
    hipEvent_t start, stop;
    bool closed;
};

std::mutex g_mu;
bool g_enabled = false;
std::vector<Record> g_records;
std::vector<hipEvent_t> g_pool;
int g_next_id = 0;  // record ids stay valid across clears (a stale id finds nothing)

hipEvent_t take_event()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

}  // namespace

bool timer_enabled()
{
    std::lock_guard<std::mutex> lk(g_mu);
    return g_enabled;
}

int timer_begin(int kernel, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_mu);
    Record r{g_next_id, kernel, take_event(), take_event(), false};
    if (r.start == nullptr || r.stop == nullptr || hipEventRecord(r.start, s) != hipSuccess) {
        if (r.start != nullptr) g_pool.push_back(r.start);
        if (r.stop != nullptr) g_pool.push_back(r.stop);
        return -1;
    }
    g_next_id = (g_next_id + 1) & 0x3fffffff;
    g_records.push_back(r);
    return r.id;
}

void timer_end(int id, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (id < 0) return;
    for (auto it = g_records.rbegin(); it != g_records.rend(); ++it) {
        if (it->id != id) continue;
        it->closed = hipEventRecord(it->stop, s) == hipSuccess;
        if (!it->closed) it->kernel = -1;  // dropped at the next read
        return;
    }
}

}  // namespace numag

using namespace numag;

extern "C" int numag_kernel_timer(int32_t enable)
{
    clear_error();
    std::lock_guard<std::mutex> lk(g_mu);
    if (enable) {
        for (const Record &r : g_records) {
            g_pool.push_back(r.start);
            g_pool.push_back(r.stop);
        }
        g_records.clear();
    }
    g_enabled = enable != 0;
    return NUMAG_OK;
}

extern "C" int numag_kernel_timer_read(int32_t kernel, double *total_ms, int64_t *launches)
{
    clear_error();
    if (kernel < 0 || kernel >= NUMAG_KERNEL_COUNT) {
        set_error("numag_kernel_timer_read: unknown kernel id");
        return NUMAG_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    double sum = 0.0;
    int64_t n = 0;
    int rc = NUMAG_OK;
    std::vector<Record> keep;
    for (const Record &r : g_records) {
        if (r.kernel == -1) {
            g_pool.push_back(r.start);
            g_pool.push_back(r.stop);
            continue;
        }
        if (r.kernel != kernel || !r.closed) {
            keep.push_back(r);  // another kernel's, or a launch still being enqueued
            continue;
        }
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(r.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.start, r.stop);
        if (e != hipSuccess && rc == NUMAG_OK) {
            set_error(std::string("numag_kernel_timer_read: ") + hipGetErrorString(e));
            rc = NUMAG_E_HIP;
        }
        sum += ms;
        ++n;
        g_pool.push_back(r.start);
        g_pool.push_back(r.stop);
    }
    g_records.swap(keep);
    if (total_ms != nullptr) *total_ms = sum;
    if (launches != nullptr) *launches = n;
    return rc;
}
