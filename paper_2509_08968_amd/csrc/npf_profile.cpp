// Kernel timing with HIP events (measurement support for the benchmark).
#include <cstring>
#include <map>

#include "npf_internal.h"

namespace npf {

hipEvent_t Profiler::take()
{
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void Profiler::clear()
{
    for (auto &r : recs) {
        pool.push_back(r.start);
        pool.push_back(r.stop);
    }
    recs.clear();
}

Profiler::~Profiler()
{
    clear();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

Timed::Timed(const npf_plan_s *p, std::string n, hipStream_t s)
    : plan(const_cast<npf_plan_s *>(p)), name(std::move(n)), stream(s)
{
    if (plan && plan->prof.on) {
        start = plan->prof.take();
        if (start) (void)hipEventRecord(start, stream);
    }
}

Timed::~Timed()
{
    if (!start) return;
    hipEvent_t stop = plan->prof.take();
    if (!stop) return;
    (void)hipEventRecord(stop, stream);
    plan->prof.recs.push_back({name, start, stop});
}

}  // namespace npf

using namespace npf;

extern "C" int npf_plan_profile(npf_plan_t plan, int32_t enable)
{
    if (!plan) return fail(NPF_E_INVALID, "null plan");
    if (enable) plan->prof.clear();
    plan->prof.on = enable != 0;
    return NPF_OK;
}

extern "C" int npf_plan_kernel_times(npf_plan_t plan, npf_kernel_time *out, int32_t capacity,
                                     int32_t *count)
{
    if (!plan || !count || (capacity > 0 && !out)) return fail(NPF_E_INVALID, "null argument");
    std::map<std::string, std::pair<int64_t, double>> agg;
    for (auto &r : plan->prof.recs) {
        if (hipEventSynchronize(r.stop) != hipSuccess)
            return fail(NPF_E_DEVICE, "event synchronisation failed");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess)
            return fail(NPF_E_DEVICE, "event timing failed");
        auto &a = agg[r.name];
        a.first += 1;
        a.second += ms;
    }
    int32_t i = 0;
    for (auto &kv : agg) {
        if (i < capacity) {
            std::memset(out[i].name, 0, sizeof(out[i].name));
            std::strncpy(out[i].name, kv.first.c_str(), sizeof(out[i].name) - 1);
            out[i].launches = kv.second.first;
            out[i].total_ms = kv.second.second;
        }
        ++i;
    }
    *count = i;
    return NPF_OK;
}
