// Process-wide HIP-event timing of one kernel class (see mbt_prof_start).
#include <mutex>
#include <vector>

#include "../../include/mbt.h"
#include "common.h"

namespace mbt {

namespace {

struct Rec {
    hipEvent_t a, b;
    double bytes, flops;
};

std::mutex g_mu;
int g_kernel = 0;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    MBT_HIP(hipEventCreate(&e));
    return e;
}

}  // namespace

ProfScope::ProfScope(int kernel, double bytes, double flops, hipStream_t st) : s_(st), bytes_(bytes), flops_(flops) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_kernel == 0 || kernel != g_kernel) return;
    a_ = take_event();
    b_ = take_event();
    MBT_HIP(hipEventRecord(a_, s_));
    on_ = true;
}

ProfScope::~ProfScope() {
    if (!on_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (hipEventRecord(b_, s_) == hipSuccess) g_recs.push_back(Rec{a_, b_, bytes_, flops_});
}

}  // namespace mbt

extern "C" {

mbt_status mbt_prof_start(int32_t kernel) {
    if (kernel < MBT_K_NONE || kernel > MBT_K_PRECOND_APPLY) return MBT_EINVAL;
    std::lock_guard<std::mutex> lk(mbt::g_mu);
    for (auto& r : mbt::g_recs) {
        (void)hipEventSynchronize(r.b);
        mbt::g_pool.push_back(r.a);
        mbt::g_pool.push_back(r.b);
    }
    mbt::g_recs.clear();
    mbt::g_kernel = kernel;
    return MBT_OK;
}

mbt_status mbt_prof_read(double* ms_total, int64_t* launches, double* bytes, double* flops) {
    std::lock_guard<std::mutex> lk(mbt::g_mu);
    double ms = 0, by = 0, fl = 0;
    for (auto& r : mbt::g_recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) return MBT_EDEVICE;
        float t = 0;
        if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return MBT_EDEVICE;
        ms += t;
        by += r.bytes;
        fl += r.flops;
    }
    if (ms_total) *ms_total = ms;
    if (launches) *launches = (int64_t)mbt::g_recs.size();
    if (bytes) *bytes = by;
    if (flops) *flops = fl;
    return MBT_OK;
}

}  // extern "C"
