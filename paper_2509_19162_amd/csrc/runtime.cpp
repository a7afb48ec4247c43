// Host runtime pieces: HIP error mapping, device buffers, look-back epochs,
// HIP-event kernel profiling.
#include <cstdio>
#include <cstring>

#include "../../include/cayleygrowth.h"
#include "internal.h"

namespace cg {

void hip_check(hipError_t e, const char *what, const char *file, int line) {
    if (e == hipSuccess) return;
    char buf[512];
    std::snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    throw Error(e == hipErrorOutOfMemory ? CG_E_NOMEM : CG_E_DEVICE, buf);
}

bool DevBuf::ensure(size_t need, double slack) {
    if (need <= bytes && p) return false;
    release();
    size_t want = (size_t)((double)need * slack);
    if (want < need) want = need;
    if (want < 256) want = 256;
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (want > need) {  // retry without slack
            want = need;
            e = hipMalloc(&q, want);
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            char buf[160];
            std::snprintf(buf, sizeof buf, "hipMalloc of %zu bytes failed", want);
            throw Error(CG_E_NOMEM, buf);
        }
    }
    p = q;
    bytes = want;
    return true;
}

void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

void PipeWork::init(hipStream_t s) {
    stream = s;
    hist.ensure(kMaxPasses * 256 * sizeof(uint64_t));
    base.ensure(kMaxPasses * 256 * sizeof(uint64_t));
    small.ensure(32 * sizeof(uint32_t) + 4 * sizeof(uint32_t) + 8 * sizeof(uint64_t) + 256);
    CG_HIP(hipMemsetAsync(small.p, 0, small.bytes, stream));
    CG_HIP(hipMemsetAsync(hist.p, 0, hist.bytes, stream));
}

void PipeWork::ensure_status(uint64_t words) {
    if (status.ensure(words * sizeof(uint64_t), 1.25)) {
        CG_HIP(hipMemsetAsync(status.p, 0, status.bytes, stream));
        epoch = 0;
    }
}

uint32_t PipeWork::next_epoch() {
    if (epoch >= 0xFFFFu) {
        CG_HIP(hipMemsetAsync(status.p, 0, status.bytes, stream));
        epoch = 0;
    }
    return ++epoch;
}

const char *kernel_kind_name(int k) {
    static const char *names[K_NUM] = {"expand",      "digit_hist", "digit_scan", "sort_pass_expand",
                                       "sort_pass",   "dedup_compact", "aux"};
    return (k >= 0 && k < K_NUM) ? names[k] : "?";
}

hipEvent_t Profiler::get_event() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e;
    CG_HIP(hipEventCreate(&e));
    return e;
}

void Profiler::begin(int kind) {
    if (!on) return;
    Pending p{kind, get_event(), get_event(), 0, 0};
    CG_HIP(hipEventRecord(p.a, stream));
    pending.push_back(p);
}

void Profiler::end(int kind, double alg_bytes, double n_items) {
    if (!on) return;
    Pending &p = pending.back();
    (void)kind;
    p.bytes = alg_bytes;
    p.items = n_items;
    CG_HIP(hipEventRecord(p.b, stream));
}

void Profiler::collect() {
    if (!on) return;
    for (auto &p : pending) {
        float ms = 0;
        CG_HIP(hipEventSynchronize(p.b));
        CG_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        total_ms[p.kind] += ms;
        bytes[p.kind] += p.bytes;
        items[p.kind] += p.items;
        launches[p.kind] += 1;
        pool.push_back(p.a);
        pool.push_back(p.b);
    }
    pending.clear();
}

Profiler::~Profiler() {
    for (auto &p : pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
}

}  // namespace cg
