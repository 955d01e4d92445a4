// Kernel timing for roofline measurement (instrumentation, not part of the
// method): HIP events recorded around launches of the FP64 update GEMM on the
// stream each launch runs on, per handle, with the launch's algorithmic flops
// and bytes.
#include "internal.h"

#include <mutex>
#include <new>
#include <vector>

namespace cdf {

struct ProfRec {
    hipEvent_t a, b;
    int kind;
    double flops, bytes;
};
struct ProfState {
    std::mutex mu;
    bool on = false;
    std::vector<ProfRec> recs;  // recs[0, used) are live; events reused across sessions
    size_t used = 0;
};

int prof_begin(ProfState *st, hipStream_t s, int kind, double flops, double bytes) {
    if (!st) return -1;
    std::lock_guard<std::mutex> lk(st->mu);
    if (!st->on) return -1;
    if (st->used == st->recs.size()) {
        ProfRec r{nullptr, nullptr, 0, 0.0, 0.0};
        if (hipEventCreate(&r.a) != hipSuccess) return -1;
        if (hipEventCreate(&r.b) != hipSuccess) { (void)hipEventDestroy(r.a); return -1; }
        st->recs.push_back(r);
    }
    ProfRec &r = st->recs[st->used];
    r.kind = kind;
    r.flops = flops;
    r.bytes = bytes;
    if (hipEventRecord(r.a, s) != hipSuccess) return -1;
    return (int)st->used++;
}

void prof_end(ProfState *st, hipStream_t s, int slot) {
    if (!st || slot < 0) return;
    std::lock_guard<std::mutex> lk(st->mu);
    if ((size_t)slot < st->used) (void)hipEventRecord(st->recs[slot].b, s);
}

hipError_t prof_enable(ProfState **pst) {
    if (!*pst) {
        *pst = new (std::nothrow) ProfState();
        if (!*pst) return hipErrorOutOfMemory;
    }
    std::lock_guard<std::mutex> lk((*pst)->mu);
    (*pst)->on = true;
    (*pst)->used = 0;
    return hipSuccess;
}

hipError_t prof_collect(ProfState *st, int kind, long long *launches, double *total_ms, double *flops,
                        double *bytes) {
    *launches = 0;
    *total_ms = 0.0;
    *flops = 0.0;
    *bytes = 0.0;
    if (!st) return hipSuccess;
    std::lock_guard<std::mutex> lk(st->mu);
    long long cnt = 0;
    double ms = 0.0, fl = 0.0, by = 0.0;
    hipError_t err = hipSuccess;
    for (size_t i = 0; i < st->used; ++i) {
        const ProfRec &r = st->recs[i];
        if (r.kind != kind) continue;
        float t = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) {
            err = hipErrorUnknown;
            continue;
        }
        ++cnt;
        ms += t;
        fl += r.flops;
        by += r.bytes;
    }
    st->on = false;  // records stay readable until the next prof_enable
    *launches = cnt;
    *total_ms = ms;
    *flops = fl;
    *bytes = by;
    return err;
}

void prof_free(ProfState *st) {
    if (!st) return;
    for (auto &r : st->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    delete st;
}

}  // namespace cdf
