// Optional per-launch timing of the sweep kernels with HIP events recorded on
// the launch stream (enabled by ct_profile_enable).
#include <mutex>
#include <vector>

#include "ct_internal.h"

namespace ct {

namespace {
struct Rec {
    int kind[4];
    double pairs;
    hipEvent_t e0, e1;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
}  // namespace

bool profiling() { return g_on; }

void* profile_begin(hipStream_t s) {
    if (!g_on) return nullptr;
    Rec r{};
    if (hipEventCreate(&r.e0) != hipSuccess || hipEventCreate(&r.e1) != hipSuccess) return nullptr;
    if (hipEventRecord(r.e0, s) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    g_recs.push_back(r);
    return reinterpret_cast<void*>(g_recs.size());
}

void profile_end(void* tok, hipStream_t s, int lagged, int bary, int code, int blocks, double pairs) {
    if (!tok) return;
    std::lock_guard<std::mutex> lk(g_mu);
    Rec& r = g_recs[reinterpret_cast<size_t>(tok) - 1];
    r.kind[0] = lagged;
    r.kind[1] = bary;
    r.kind[2] = code;
    r.kind[3] = blocks;
    r.pairs = pairs;
    (void)hipEventRecord(r.e1, s);
}

void* profile_kernel_begin(hipEvent_t* e0, hipEvent_t* e1) {
    *e0 = *e1 = nullptr;
    if (!g_on) return nullptr;
    Rec r{};
    if (hipEventCreate(&r.e0) != hipSuccess) return nullptr;
    if (hipEventCreate(&r.e1) != hipSuccess) {
        (void)hipEventDestroy(r.e0);
        return nullptr;
    }
    *e0 = r.e0;
    *e1 = r.e1;
    std::lock_guard<std::mutex> lk(g_mu);
    g_recs.push_back(r);
    return reinterpret_cast<void*>(g_recs.size());
}

void profile_kernel_end(void* tok, int lagged, int bary, int code, int blocks, double pairs) {
    if (!tok) return;
    std::lock_guard<std::mutex> lk(g_mu);
    Rec& r = g_recs[reinterpret_cast<size_t>(tok) - 1];
    r.kind[0] = lagged;
    r.kind[1] = bary;
    r.kind[2] = code;
    r.kind[3] = blocks;
    r.pairs = pairs;
}

}  // namespace ct

using namespace ct;

extern "C" ct_status ct_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_on = on != 0;
    return CT_OK;
}

extern "C" int32_t ct_profile_count(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    return (int32_t)g_recs.size();
}

extern "C" ct_status ct_profile_read(int32_t i, int32_t* kind4, double* pairs, float* ms) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (i < 0 || i >= (int32_t)g_recs.size()) return fail(CT_E_ARG, "record %d out of range", i);
    Rec& r = g_recs[i];
    CT_CHECK_HIP(hipEventSynchronize(r.e1));
    float t = 0.f;
    CT_CHECK_HIP(hipEventElapsedTime(&t, r.e0, r.e1));
    if (kind4)
        for (int k = 0; k < 4; ++k) kind4[k] = r.kind[k];
    if (pairs) *pairs = r.pairs;
    if (ms) *ms = t;
    return CT_OK;
}

extern "C" void ct_profile_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& r : g_recs) {
        (void)hipEventDestroy(r.e0);
        (void)hipEventDestroy(r.e1);
    }
    g_recs.clear();
}
