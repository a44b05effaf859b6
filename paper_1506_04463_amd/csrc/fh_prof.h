// Optional per-kernel timing with HIP events (enabled per handle).  Launchers
// bracket their main kernel with prof_begin/prof_end; with profiling off both
// are no-ops.  Pending event pairs are resolved when the statistics are read.
#pragma once
#include <map>
#include <string>
#include <vector>

#include "fh_common.h"

namespace fh {

struct Prof {
    struct Pending {
        hipEvent_t a, b;
        std::string name;
        double bytes, flops;
    };
    struct Stat {
        long long count = 0;
        double ms = 0.0, bytes = 0.0, flops = 0.0;
    };
    std::vector<Pending> pend;
    std::vector<hipEvent_t> pool;
    std::map<std::string, Stat> stats;
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        FH_HIP(hipEventCreate(&e));
        return e;
    }
    void resolve() {
        for (auto& p : pend) {
            FH_HIP(hipEventSynchronize(p.b));
            float ms = 0.f;
            FH_HIP(hipEventElapsedTime(&ms, p.a, p.b));
            Stat& s = stats[p.name];
            s.count++;
            s.ms += ms;
            s.bytes += p.bytes;
            s.flops += p.flops;
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pend.clear();
    }
    void reset() {
        resolve();
        stats.clear();
    }
    ~Prof() {
        for (auto& p : pend) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

// the profiler of the handle currently executing on this thread (or null)
inline Prof*& tl_prof() {
    static thread_local Prof* p = nullptr;
    return p;
}

inline hipEvent_t prof_begin(hipStream_t st) {
    Prof* p = tl_prof();
    if (!p) return nullptr;
    hipEvent_t e = p->get();
    FH_HIP(hipEventRecord(e, st));
    return e;
}

inline void prof_end(hipStream_t st, hipEvent_t a, const std::string& name, double bytes, double flops = 0.0) {
    Prof* p = tl_prof();
    if (!p || !a) return;
    hipEvent_t b = p->get();
    FH_HIP(hipEventRecord(b, st));
    p->pend.push_back({a, b, name, bytes, flops});
    if (p->pend.size() > 4096) p->resolve();
}

}  // namespace fh
