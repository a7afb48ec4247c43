// Host runtime pieces: HIP error mapping, device buffers, look-back epochs,
// HIP-event kernel profiling.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <iterator>
#include <cstring>
#include <map>
#include <mutex>

#include "../../include/cayleygrowth.h"
#include "internal.h"

namespace cg {

void hip_check(hipError_t e, const char *what, const char *file, int line) {
    if (e == hipSuccess) return;
    char buf[512];
    std::snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    throw Error(e == hipErrorOutOfMemory ? CG_E_NOMEM : CG_E_DEVICE, buf);
}

// ---------------------------------------------------------------------------
// Device arena. On this HIP runtime a hipMalloc is fast while little memory is
// held, but a large one takes seconds once tens of GB are already held. So
// the first large request reserves one big region (CG_ARENA_FRACTION of the
// free memory, default 0.85; 0 disables it) and every buffer is carved out
// of it: best fit, split on allocation, coalesced on free. A range is
// freed only after its owner's stream has drained, so work still queued on
// the old stream never races with a new owner. Requests the arena cannot
// hold fall back to plain hipMalloc/hipFree.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kAlign = 1u << 16;
constexpr size_t kArenaMinRequest = 64u << 20;  // smaller buffers also use it once it exists

struct Arena {
    char *base = nullptr;
    size_t size = 0;
    bool tried = false;
    bool external = false;  // the caller's memory (cg_set_workspace): never freed here
    std::map<size_t, size_t> by_off;            // free ranges: offset -> length
    std::multimap<size_t, size_t> by_len;       // free ranges: length -> offset
    size_t used = 0;

    void insert_free(size_t off, size_t len) {
        auto nx = by_off.lower_bound(off);
        if (nx != by_off.end() && off + len == nx->first) {  // merge with the next range
            erase_len(nx->second, nx->first);
            len += nx->second;
            nx = by_off.erase(nx);
        }
        if (nx != by_off.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {  // merge with the previous range
                erase_len(pv->second, pv->first);
                off = pv->first;
                len += pv->second;
                by_off.erase(pv);
            }
        }
        by_off[off] = len;
        by_len.emplace(len, off);
    }
    void erase_len(size_t len, size_t off) {
        auto r = by_len.equal_range(len);
        for (auto it = r.first; it != r.second; ++it)
            if (it->second == off) {
                by_len.erase(it);
                return;
            }
    }
    bool take(size_t len, size_t &off) {
        auto it = by_len.lower_bound(len);
        if (it == by_len.end()) return false;
        const size_t flen = it->first, foff = it->second;
        by_len.erase(it);
        by_off.erase(foff);
        if (flen > len) insert_free(foff + len, flen - len);
        off = foff;
        used += len;
        return true;
    }
};

struct DeviceArenas {
    std::mutex mu;
    std::map<int, Arena> arena;
};

DeviceArenas &arenas() {
    static DeviceArenas *a = new DeviceArenas();  // never destroyed: outlives every user
    return *a;
}

int current_device() {
    int d = 0;
    (void)hipGetDevice(&d);
    return d;
}

double arena_fraction() {
    const char *e = std::getenv("CG_ARENA_FRACTION");
    if (!e) return 0.85;
    const double f = std::atof(e);
    return f < 0 ? 0 : (f > 0.95 ? 0.95 : f);
}

// Returns a pointer inside the device's arena, or nullptr.
void *arena_alloc(int dev, size_t len) {
    std::lock_guard<std::mutex> lk(arenas().mu);
    Arena &A = arenas().arena[dev];
    if (!A.base) {
        if (A.tried || len < kArenaMinRequest) return nullptr;
        A.tried = true;
        const double frac = arena_fraction();
        size_t free_b = 0, total_b = 0;
        if (frac <= 0 || hipMemGetInfo(&free_b, &total_b) != hipSuccess) return nullptr;
        size_t want = (size_t)((double)free_b * frac) / kAlign * kAlign;
        void *p = nullptr;
        if (want < len || hipMalloc(&p, want) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        A.base = (char *)p;
        A.size = want;
        A.insert_free(0, want);
    }
    size_t off = 0;
    if (!A.take(len, off)) return nullptr;
    return A.base + off;
}

bool arena_free(int dev, void *p, size_t len) {
    std::lock_guard<std::mutex> lk(arenas().mu);
    auto it = arenas().arena.find(dev);
    if (it == arenas().arena.end() || !it->second.base) return false;
    Arena &A = it->second;
    char *c = (char *)p;
    if (c < A.base || c >= A.base + A.size) return false;
    A.insert_free((size_t)(c - A.base), len);
    A.used -= len;
    return true;
}

}  // namespace

void release_cached_device_memory() {
    std::lock_guard<std::mutex> lk(arenas().mu);
    for (auto &kv : arenas().arena) {
        Arena &A = kv.second;
        if (!A.base || A.used || A.external) continue;  // in use, or the caller's
        (void)hipFree(A.base);
        A = Arena{};
    }
}

void set_workspace(void *p, size_t bytes) {
    const int dev = current_device();
    std::lock_guard<std::mutex> lk(arenas().mu);
    Arena &A = arenas().arena[dev];
    if (A.base && A.used) throw Error(CG_E_BUSY, "device buffers still live in the current workspace");
    if (A.base && !A.external) (void)hipFree(A.base);
    A = Arena{};
    if (!p) return;  // back to memory the library reserves itself
    const uintptr_t lo = ((uintptr_t)p + 255) & ~(uintptr_t)255;
    const size_t skip = (size_t)(lo - (uintptr_t)p);
    if (bytes <= skip + kAlign) throw Error(CG_E_INVAL, "workspace smaller than 64 KiB");
    const size_t size = (bytes - skip) / kAlign * kAlign;
    A.base = (char *)lo;
    A.size = size;
    A.external = true;
    A.tried = true;
    A.insert_free(0, size);
}

bool arena_active() {
    const int dev = current_device();
    std::lock_guard<std::mutex> lk(arenas().mu);
    auto it = arenas().arena.find(dev);
    return it != arenas().arena.end() && it->second.base;
}

size_t device_bytes_available() {
    const int dev = current_device();
    {
        std::lock_guard<std::mutex> lk(arenas().mu);
        auto it = arenas().arena.find(dev);
        if (it != arenas().arena.end() && it->second.base) {
            const auto &by_len = it->second.by_len;
            return by_len.empty() ? 0 : by_len.rbegin()->first;
        }
    }
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return free_b;
}

namespace {
// bytes held by every DevBuf of the process (all devices), and the most
// they held at once since the last reset
std::atomic<uint64_t> g_held{0}, g_peak_held{0};

void count_held(uint64_t add) {
    const uint64_t now = g_held.fetch_add(add) + add;
    uint64_t pk = g_peak_held.load();
    while (now > pk && !g_peak_held.compare_exchange_weak(pk, now)) {
    }
}
}  // namespace

void memory_stats(cg_memory_stats_t *out, bool reset_peak) {
    out->held_bytes = g_held.load();
    out->peak_held_bytes = g_peak_held.load();
    uint64_t reserved = 0;
    {
        std::lock_guard<std::mutex> lk(arenas().mu);
        for (auto &kv : arenas().arena)
            if (kv.second.base && !kv.second.external) reserved += kv.second.size;
    }
    out->arena_bytes = reserved;
    if (reset_peak) g_peak_held.store(g_held.load());
}

bool DevBuf::ensure(size_t need, double slack) {
    if (need <= bytes && p) return false;
    const size_t old = bytes;
    release();
    size_t want = (size_t)((double)need * slack);
    if (want < need) want = need;
    if (old && want < old + old / 2) want = std::max(need, old + old / 2);  // grow geometrically
    if (arena_active()) want = need;  // re-carving the arena is cheap: no slack
    want = (std::max<size_t>(want, 256) + kAlign - 1) / kAlign * kAlign;
    dev = current_device();
    void *q = arena_alloc(dev, want);
    if (q) {
        in_arena = true;
    } else {
        in_arena = false;
        hipError_t e = hipMalloc(&q, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            want = (need + kAlign - 1) / kAlign * kAlign;  // retry without slack
            e = hipMalloc(&q, want);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                char buf[160];
                std::snprintf(buf, sizeof buf, "device allocation of %zu bytes failed", want);
                throw Error(CG_E_NOMEM, buf);
            }
        }
    }
    p = q;
    bytes = want;
    count_held(want);
    return true;
}

void DevBuf::release() {
    if (p) {
        if (in_arena) {
            // Work still queued on the owner stream may use the range: wait
            // for it, then hand the range back. (No event is kept for later:
            // the owner stream may be destroyed before anyone would query it.)
            if (hipStreamSynchronize(stream) != hipSuccess) {
                (void)hipGetLastError();
                (void)hipDeviceSynchronize();
            }
            (void)arena_free(dev, p, bytes);
        } else {
            (void)hipFree(p);  // a block of its own; synchronises the device
        }
        g_held.fetch_sub(bytes);
    }
    p = nullptr;
    bytes = 0;
}

void PipeWork::init(hipStream_t s) {
    stream = s;
    for (DevBuf *b : {&hist, &base, &small, &status, &bounds, &tile_cnt, &tile_off, &kill, &tcnt, &toff, &bsum})
        b->stream = s;
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
