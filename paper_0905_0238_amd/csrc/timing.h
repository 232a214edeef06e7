// Optional per-kernel timing with HIP events, for benchmarks and profiling.
// When enabled on a plan, each kernel launch made for that plan is bracketed
// by two events recorded on the launch stream; edt_timing_read sums the
// elapsed times per kernel name.  Disabled (the default) it costs nothing.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

struct edt_plan;

namespace edt {

struct TimerRec {
    const char* name;
    hipEvent_t start, stop;
};

struct Timer {
    bool enabled = false;
    std::vector<TimerRec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t pending = nullptr;

    hipEvent_t take() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void begin(hipStream_t st) {
        if (!enabled) return;
        pending = take();
        if (pending) (void)hipEventRecord(pending, st);
    }
    void end(hipStream_t st, const char* name) {
        if (!enabled || !pending) return;
        hipEvent_t e = take();
        if (!e) return;
        (void)hipEventRecord(e, st);
        recs.push_back(TimerRec{name, pending, e});
        pending = nullptr;
    }
    ~Timer() {
        for (auto& r : recs) {
            (void)hipEventDestroy(r.start);
            (void)hipEventDestroy(r.stop);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

Timer& timer_of(const edt_plan* p);

}  // namespace edt
