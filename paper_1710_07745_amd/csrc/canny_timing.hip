// Per-stage device timing: HIP event pairs recorded on the caller's stream
// around the kernels of one stage, summed on request.  Off by default; when
// off, a stage costs one relaxed atomic load on the host.
#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/canny.h"
#include "canny_internal.h"

namespace canny {
namespace {

struct StagePool {
    std::vector<hipEvent_t> a, b;
    int used = 0;
};

std::mutex g_mu;
std::atomic<bool> g_on{false};
int g_cap = 0;
StagePool g_pool[CANNY_STAGE_COUNT];

void destroy_locked() {
    g_on.store(false, std::memory_order_relaxed);
    for (auto& p : g_pool) {
        for (hipEvent_t e : p.a) (void)hipEventDestroy(e);
        for (hipEvent_t e : p.b) (void)hipEventDestroy(e);
        p.a.clear();
        p.b.clear();
        p.used = 0;
    }
    g_cap = 0;
}

}  // namespace

int timing_begin(int stage, hipStream_t s) {
    if (!g_on.load(std::memory_order_relaxed)) return -1;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on.load(std::memory_order_relaxed)) return -1;
    StagePool& p = g_pool[stage];
    if (p.used >= g_cap) return -1;
    const int slot = p.used++;
    (void)hipEventRecord(p.a[slot], s);
    return slot;
}

void timing_end(int stage, int slot, hipStream_t s) {
    if (slot < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on.load(std::memory_order_relaxed)) return;
    (void)hipEventRecord(g_pool[stage].b[slot], s);
}

}  // namespace canny

using namespace canny;

extern "C" {

int canny_timing_begin(int capacity) {
    if (capacity < 1 || capacity > 65536) return CANNY_ERR_INVALID;
    std::lock_guard<std::mutex> lk(g_mu);
    destroy_locked();
    for (auto& p : g_pool) {
        p.a.resize(capacity);
        p.b.resize(capacity);
        for (int i = 0; i < capacity; ++i) {
            if (hipEventCreate(&p.a[i]) != hipSuccess || hipEventCreate(&p.b[i]) != hipSuccess) {
                p.a.resize(i);  // keep only created pairs for destruction
                p.b.resize(i);
                destroy_locked();
                return CANNY_ERR_HIP;
            }
        }
    }
    g_cap = capacity;
    g_on.store(true, std::memory_order_relaxed);
    return CANNY_OK;
}

int canny_timing_read(int stage, double* ms_total, int64_t* launches) {
    if (stage < 0 || stage >= CANNY_STAGE_COUNT || !ms_total || !launches) return CANNY_ERR_INVALID;
    std::lock_guard<std::mutex> lk(g_mu);
    const StagePool& p = g_pool[stage];
    double sum = 0.0;
    for (int i = 0; i < p.used; ++i) {
        if (hipEventSynchronize(p.b[i]) != hipSuccess) return CANNY_ERR_HIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.a[i], p.b[i]) != hipSuccess) return CANNY_ERR_HIP;
        sum += ms;
    }
    *ms_total = sum;
    *launches = p.used;
    return CANNY_OK;
}

int canny_timing_end(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    destroy_locked();
    return CANNY_OK;
}

}  // extern "C"
