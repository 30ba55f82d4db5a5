// HIP-event timing of selected kernel launches (wl_profile_*): each timed
// launch is bracketed by two events on its own stream; totals are summed when
// read.  Events come from a process-wide pool that grows on demand.
#include <atomic>
#include <mutex>
#include <vector>

#include "wl_internal.h"

namespace wl {
namespace {

struct Rec {
    hipEvent_t a, b;
};

struct Profiler {
    std::mutex mu;
    std::atomic<unsigned> mask{0};
    std::vector<Rec> pending[WL_PROF_COUNT];
    std::vector<Rec> pool;
    double total_ms[WL_PROF_COUNT] = {};
    long long launches[WL_PROF_COUNT] = {};
    long long cells[WL_PROF_COUNT] = {};

    Rec get() {
        if (!pool.empty()) {
            Rec r = pool.back();
            pool.pop_back();
            return r;
        }
        Rec r{};
        (void)hipEventCreate(&r.a);
        (void)hipEventCreate(&r.b);
        return r;
    }
};

Profiler& prof() {
    static Profiler p;
    return p;
}

thread_local Rec t_open[WL_PROF_COUNT];

}  // namespace

// Timing of a kernel that runs inside captured solve bodies (the multigrid
// sweeps and transfers) turns graph replay off.
bool prof_active() {
    constexpr unsigned in_graphs = (1u << WL_PROF_SMOOTH_FINE) | (1u << WL_PROF_SMOOTH_NORM) |
                                   (1u << WL_PROF_PROLONG_FINE) | (1u << WL_PROF_RESTRICT_FINE) |
                                   (1u << WL_PROF_NORM_FINE) | (1u << WL_PROF_PAIR_FINE) |
                                   (1u << WL_PROF_PAIR_PROLONG_FINE);
    return (prof().mask.load(std::memory_order_relaxed) & in_graphs) != 0u;
}

namespace {
std::atomic<int> g_graphs{1};
}  // namespace

bool graphs_enabled() { return g_graphs.load(std::memory_order_relaxed) != 0; }

GraphCache::~GraphCache() {
    for (auto& en : e)
        if (en.exec) (void)hipGraphExecDestroy(en.exec);
    if (cap) (void)hipStreamDestroy(cap);
}

void GraphCache::clear() {
    for (auto& en : e) {
        if (en.exec) (void)hipGraphExecDestroy(en.exec);
        en = Entry{};
    }
}

ProfScope::ProfScope(int kernel, hipStream_t stream, size_t ncells) : id(kernel), s(stream) {
    Profiler& P = prof();
    on = kernel >= 0 && kernel < WL_PROF_COUNT && (P.mask.load() >> kernel & 1u);
    if (!on) return;
    std::lock_guard<std::mutex> g(P.mu);
    Rec r = P.get();
    t_open[kernel] = r;
    P.cells[kernel] = (long long)ncells;
    (void)hipEventRecord(r.a, stream);
}

ProfScope::~ProfScope() {
    if (!on) return;
    Profiler& P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    Rec r = t_open[id];
    (void)hipEventRecord(r.b, s);
    P.pending[id].push_back(r);
}

static void drain(Profiler& P, int k) {
    for (Rec& r : P.pending[k]) {
        float ms = 0.f;
        (void)hipEventSynchronize(r.b);
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            P.total_ms[k] += ms;
            P.launches[k] += 1;
        }
        P.pool.push_back(r);
    }
    P.pending[k].clear();
}

}  // namespace wl

using namespace wl;

extern "C" {

wl_status wl_set_graphs(int enable) {
    clear_error();
    g_graphs.store(enable != 0 ? 1 : 0, std::memory_order_relaxed);
    return WL_OK;
}

wl_status wl_profile_enable(unsigned mask) {
    clear_error();
    Profiler& P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    P.mask.store(mask);
    return WL_OK;
}

wl_status wl_profile_reset(void) {
    clear_error();
    Profiler& P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    for (int k = 0; k < WL_PROF_COUNT; ++k) {
        drain(P, k);
        P.total_ms[k] = 0.0;
        P.launches[k] = 0;
    }
    return WL_OK;
}

wl_status wl_profile_read(int kernel, double* total_ms, long long* launches,
                          long long* cells_per_launch) {
    clear_error();
    if (kernel < 0 || kernel >= WL_PROF_COUNT) {
        set_error("unknown kernel id");
        return WL_ERR_INVALID_ARG;
    }
    Profiler& P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    drain(P, kernel);
    if (total_ms) *total_ms = P.total_ms[kernel];
    if (launches) *launches = P.launches[kernel];
    if (cells_per_launch) *cells_per_launch = P.cells[kernel];
    return WL_OK;
}

}  // extern "C"
