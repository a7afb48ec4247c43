// Growth over rank-space bitmaps: the small-job engine (one workgroup per
// job, one persistent launch for a whole batch) and the bitmask engine (one
// job over the whole device, 3 bits per state). The layer rule is the
// breadth-first one of the definition of growth (paper, section "Reminder
// on Cayley graphs, diameters, growth"): layer d+1 holds the neighbours
// s.g of layer d that no earlier layer holds. A visited bitmap stands for
// "every earlier layer", so no closure under inverses is assumed.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>

#include "bitmap.h"
#include "device_util.h"
#include "expand_device.h"
#include "internal.h"
#include "perm_rank.h"

// Device memory of cg_growth_batch_noalloc: every buffer its launch needs
// beyond the caller's inputs and outputs (job table, generator table,
// layer-size and outcome staging, the job-queue tickets, the per-workgroup
// bitmap slots of n = 9, 10 jobs). Each GPU the library runs on holds its
// own copy until the process ends. Host code never uses this name as an
// address: it takes the device address once per device from
// hipGetSymbolAddress (cg::noalloc_scratch).
constexpr size_t kNoAllocScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace cg {

namespace {

__host__ __device__ constexpr uint64_t factorial(int n) { return n <= 1 ? 1ull : (uint64_t)n * factorial(n - 1); }

template <int N>
using RankOf = typename std::conditional<(N <= 12), uint32_t, uint64_t>::type;

// Lexicographic rank on the host for any n <= 16 (64-bit).
uint64_t host_rank64(uint64_t key, int n) {
    uint64_t rank = 0;
    uint32_t used = 0;
    for (int i = 0; i < n; ++i) {
        const uint32_t v = (uint32_t)(key >> (4 * (n - 1 - i))) & 15u;
        const uint32_t c = v - (uint32_t)__builtin_popcount(used & ((1u << v) - 1u));
        rank = rank * (uint64_t)(n - i) + c;
        used |= 1u << v;
    }
    return rank;
}

// Release this workgroup's writes to device memory, wait for all its
// waves, then drop stale L1 lines: bitmap words change by L2 atomics.
__device__ __forceinline__ void wg_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// ---------------------------------------------------------------------------
// Small-job engine
// ---------------------------------------------------------------------------
struct WgJobDev {
    uint32_t n, k, goff, start_rank;
    uint32_t max_layers, pad;
    uint64_t max_frontier;  // 0 = none
    uint64_t sizes_off;     // first entry of the job's layer sizes
};
struct WgOutDev {
    int32_t status, num_layers;
    uint64_t expanded;
};

constexpr uint32_t kWgLdsN = 8;
constexpr uint32_t kWgLdsWords = (uint32_t)((factorial(kWgLdsN) + 31) / 32);  // 1260
constexpr int kWgMaxBlock = 1024;

template <int N>
__device__ __forceinline__ void wg_run(const WgJobDev &J, const GenSel *__restrict__ gtab, uint32_t *vis,
                                       uint32_t *cur, uint32_t *nxt, uint64_t *__restrict__ sizes,
                                       WgOutDev *__restrict__ out, GenSel *s_sel, uint32_t *s_acc) {
    constexpr uint32_t W = (uint32_t)((factorial(N) + 31) / 32);
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const int k = (int)J.k;
    for (uint32_t i = tid; i < (uint32_t)k * 8u; i += nt) (&s_sel[0].sel[0])[i] = (&gtab[J.goff].sel[0])[i];
    for (uint32_t w = tid; w < W; w += nt) {
        vis[w] = 0u;
        cur[w] = 0u;
        nxt[w] = 0u;
    }
    wg_barrier();
    if (tid == 0) {
        const uint32_t r = J.start_rank;
        vis[r >> 5] = 1u << (r & 31u);
        cur[r >> 5] = 1u << (r & 31u);
        sizes[0] = 1;
    }
    wg_barrier();
    uint64_t F = 1, expanded = 0;
    uint32_t layers = 1;
    int status = CG_OK;
    for (;;) {
        if (k == 0) break;
        if (J.max_frontier && F > J.max_frontier) {
            status = CG_TRUNCATED;
            break;
        }
        if (layers >= J.max_layers) {
            status = CG_TRUNCATED;
            break;
        }
        // expand layer d: every set bit of cur, every generator
        for (uint32_t w = tid; w < W; w += nt) {
            uint32_t bits = cur[w];
            while (bits) {
                const uint32_t b = (uint32_t)__builtin_ctz(bits);
                bits &= bits - 1u;
                const Nibbles s = split_nibbles(perm_unrank_t<N>(w * 32u + b));
                for (int g = 0; g < k; ++g) {
                    const uint32_t q = perm_rank_t<N>(apply_gensel(s, s_sel[g]));
                    const uint32_t m = 1u << (q & 31u);
                    if (!(vis[q >> 5] & m)) atomicOr(&nxt[q >> 5], m);
                }
            }
        }
        if (tid == 0) *s_acc = 0;
        wg_barrier();
        // fold: visited |= next, count it, clear the expanded layer
        uint32_t cnt = 0;
        for (uint32_t w = tid; w < W; w += nt) {
            const uint32_t x = nxt[w];
            if (x) {
                vis[w] |= x;
                cnt += (uint32_t)__popc(x);
            }
            cur[w] = 0u;
        }
        cnt = wave_sum(cnt);
        if ((tid & (kWave - 1)) == 0 && cnt) atomicAdd(s_acc, cnt);
        wg_barrier();
        const uint32_t n1 = *s_acc;
        expanded += F;
        uint32_t *t = cur;
        cur = nxt;
        nxt = t;
        if (n1 == 0) break;
        if (tid == 0) sizes[layers] = n1;
        ++layers;
        F = n1;
        wg_barrier();  // every thread has read s_acc before it is reset
    }
    if (tid == 0) {
        out->status = status;
        out->num_layers = (int32_t)layers;
        out->expanded = expanded;
    }
}

// One persistent launch for a whole batch: each workgroup takes the next
// job from a queue (jobs are ordered by decreasing size) and runs it to
// completion. Jobs with n >= 9 use the workgroup's slot of `gbits`
// (3 * slot_words words, checked by the host to hold their bitmaps); only
// workgroups below n_slot_blocks own a slot. Two queues: ticket[0] hands
// out jobs [0, n_slot_jobs) to workgroups that own a slot, ticket[1] jobs
// [n_slot_jobs, njobs) to every workgroup (the host puts a job with
// n >= 9 there only when every workgroup owns a slot).
__global__ __launch_bounds__(kWgMaxBlock) void wg_growth_kernel(const WgJobDev *__restrict__ jobs, uint32_t njobs,
                                                                uint32_t n_slot_jobs, uint32_t n_slot_blocks,
                                                                const GenSel *__restrict__ gtab,
                                                                uint64_t *__restrict__ sizes,
                                                                WgOutDev *__restrict__ outs, uint32_t *ticket,
                                                                uint32_t *gbits, uint64_t slot_words) {
    __shared__ uint32_t s_bits[3 * kWgLdsWords];
    __shared__ GenSel s_sel[kBitmapMaxK];
    __shared__ uint32_t s_acc, s_job;
    const bool has_slot = gbits && blockIdx.x < n_slot_blocks;
    uint32_t *slot = has_slot ? gbits + (uint64_t)blockIdx.x * 3ull * slot_words : nullptr;
    for (uint32_t q = has_slot ? 0u : 1u; q < 2u; ++q) {
    const uint32_t q_lo = q ? n_slot_jobs : 0u, q_hi = q ? njobs : n_slot_jobs;
    for (;;) {
        if (threadIdx.x == 0) s_job = atomicAdd(ticket + q, 1u);
        __syncthreads();
        const uint32_t t = s_job;
        __syncthreads();
        if (t >= q_hi - q_lo) break;
        const uint32_t j = q_lo + t;
        const WgJobDev J = jobs[j];
        if (J.n > kWgLdsN && !slot) {
            // a host bookkeeping error: report it instead of touching memory
            if (threadIdx.x == 0) {
                outs[j].status = CG_E_DEVICE;
                outs[j].num_layers = 0;
                outs[j].expanded = 0;
            }
            continue;
        }
        uint64_t *sz = sizes + J.sizes_off;
        uint32_t *l0 = s_bits, *l1 = s_bits + kWgLdsWords, *l2 = s_bits + 2 * kWgLdsWords;
        switch (J.n) {
            case 1: wg_run<1>(J, gtab, l0, l1, l2, sz, outs + j, s_sel, &s_acc); break;
            case 2: wg_run<2>(J, gtab, l0, l1, l2, sz, outs + j, s_sel, &s_acc); break;
            case 3: wg_run<3>(J, gtab, l0, l1, l2, sz, outs + j, s_sel, &s_acc); break;
            case 4: wg_run<4>(J, gtab, l0, l1, l2, sz, outs + j, s_sel, &s_acc); break;
            case 5: wg_run<5>(J, gtab, l0, l1, l2, sz, outs + j, s_sel, &s_acc); break;
            case 6: wg_run<6>(J, gtab, l0, l1, l2, sz, outs + j, s_sel, &s_acc); break;
            case 7: wg_run<7>(J, gtab, l0, l1, l2, sz, outs + j, s_sel, &s_acc); break;
            case 8: wg_run<8>(J, gtab, l0, l1, l2, sz, outs + j, s_sel, &s_acc); break;
            case 9:
                wg_run<9>(J, gtab, slot, slot + slot_words, slot + 2 * slot_words, sz, outs + j, s_sel, &s_acc);
                break;
            default:
                wg_run<10>(J, gtab, slot, slot + slot_words, slot + 2 * slot_words, sz, outs + j, s_sel, &s_acc);
                break;
        }
        __syncthreads();
    }
    }
}

__global__ void clear_u32_kernel(uint32_t *p, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------------------
// Bitmask engine (one job, whole device)
// ---------------------------------------------------------------------------
constexpr uint32_t kChunkWords = 1024;  // bitmap words per summary bit
constexpr int kBmBlock = 256;

template <int N>
__global__ __launch_bounds__(kBmBlock) void bm_expand_kernel(const uint32_t *__restrict__ cur,
                                                             const uint32_t *__restrict__ scur,
                                                             const uint32_t *__restrict__ vis, uint32_t *nxt,
                                                             uint32_t *snxt, uint64_t W, uint64_t nchunks,
                                                             const GenSel *__restrict__ gsel, int k) {
    using R = RankOf<N>;
    __shared__ GenSel s_sel[kBitmapMaxK];
    for (int i = threadIdx.x; i < k * 8; i += kBmBlock) (&s_sel[0].sel[0])[i] = (&gsel[0].sel[0])[i];
    __syncthreads();
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        if (!((scur[c >> 5] >> (c & 31u)) & 1u)) continue;  // no state of layer d here
        const uint64_t w_end = (c + 1) * kChunkWords < W ? (c + 1) * kChunkWords : W;
        for (uint64_t w = c * kChunkWords + threadIdx.x; w < w_end; w += kBmBlock) {
            uint32_t bits = cur[w];
            while (bits) {
                const uint32_t b = (uint32_t)__builtin_ctz(bits);
                bits &= bits - 1u;
                const Nibbles s = split_nibbles(perm_unrank_t<N, R>((R)(w * 32u + b)));
                for (int g = 0; g < k; ++g) {
                    const uint64_t q = (uint64_t)perm_rank_t<N, R>(apply_gensel(s, s_sel[g]));
                    const uint64_t qw = q >> 5;
                    const uint32_t m = 1u << (uint32_t)(q & 31u);
                    if (vis[qw] & m) continue;
                    if (nxt[qw] & m) continue;  // may read stale: then the atomic below decides
                    const uint32_t old = atomicOr(&nxt[qw], m);
                    if (old == 0u) {  // first bit of this word in layer d+1: mark its chunk
                        const uint64_t qc = qw / kChunkWords;
                        atomicOr(&snxt[qc >> 5], 1u << (uint32_t)(qc & 31u));
                    }
                }
            }
        }
    }
}

// visited |= next (counted), and the expanded layer is cleared, over the
// chunks that either touches.
__global__ __launch_bounds__(kBmBlock) void bm_fold_kernel(uint32_t *__restrict__ vis, uint32_t *__restrict__ cur,
                                                           const uint32_t *__restrict__ scur,
                                                           const uint32_t *__restrict__ nxt,
                                                           const uint32_t *__restrict__ snxt, uint64_t W,
                                                           uint64_t nchunks, unsigned long long *count) {
    __shared__ uint32_t s_acc;
    if (threadIdx.x == 0) s_acc = 0;
    __syncthreads();
    uint32_t cnt = 0;
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const bool in_next = (snxt[c >> 5] >> (c & 31u)) & 1u;
        const bool in_cur = (scur[c >> 5] >> (c & 31u)) & 1u;
        if (!in_next && !in_cur) continue;
        const uint64_t w_end = (c + 1) * kChunkWords < W ? (c + 1) * kChunkWords : W;
        for (uint64_t w = c * kChunkWords + threadIdx.x; w < w_end; w += kBmBlock) {
            if (in_next) {
                const uint32_t x = nxt[w];
                if (x) {
                    vis[w] |= x;
                    cnt += (uint32_t)__popc(x);
                }
            }
            if (in_cur) cur[w] = 0u;
        }
    }
    cnt = wave_sum(cnt);
    if ((threadIdx.x & (kWave - 1)) == 0 && cnt) atomicAdd(&s_acc, cnt);
    __syncthreads();
    if (threadIdx.x == 0 && s_acc) atomicAdd(count, (unsigned long long)s_acc);
}

__global__ void bm_seed_kernel(uint32_t *vis, uint32_t *cur, uint32_t *scur, uint64_t r,
                               unsigned long long *count) {
    const uint64_t w = r >> 5;
    const uint32_t m = 1u << (uint32_t)(r & 31u);
    vis[w] = m;
    cur[w] = m;
    const uint64_t c = w / kChunkWords;
    scur[c >> 5] = 1u << (uint32_t)(c & 31u);
    *count = 0;
}

__global__ void bm_clear_kernel(uint32_t *a, uint64_t na, unsigned long long *count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na; i += (uint64_t)gridDim.x * blockDim.x)
        a[i] = 0u;
    if (count && blockIdx.x == 0 && threadIdx.x == 0) *count = 0;
}

template <class F>
void with_bm_n(int n, F &&f) {
    switch (n) {
        case 1: f(std::integral_constant<int, 1>{}); break;
        case 2: f(std::integral_constant<int, 2>{}); break;
        case 3: f(std::integral_constant<int, 3>{}); break;
        case 4: f(std::integral_constant<int, 4>{}); break;
        case 5: f(std::integral_constant<int, 5>{}); break;
        case 6: f(std::integral_constant<int, 6>{}); break;
        case 7: f(std::integral_constant<int, 7>{}); break;
        case 8: f(std::integral_constant<int, 8>{}); break;
        case 9: f(std::integral_constant<int, 9>{}); break;
        case 10: f(std::integral_constant<int, 10>{}); break;
        case 11: f(std::integral_constant<int, 11>{}); break;
        case 12: f(std::integral_constant<int, 12>{}); break;
        case 13: f(std::integral_constant<int, 13>{}); break;
        default: f(std::integral_constant<int, 14>{}); break;
    }
}

int device_cus() {
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    return cus;
}

}  // namespace

bool start_is_permutation(const JobSpec &spec) {
    bool seen[16] = {false};
    for (int i = 0; i < spec.n; ++i) {
        if (spec.start[i] >= spec.n || seen[spec.start[i]]) return false;
        seen[spec.start[i]] = true;
    }
    return true;
}

bool wg_eligible(const JobSpec &spec) {
    return spec.n <= kWgMaxN && spec.k <= kBitmapMaxK && start_is_permutation(spec) && !spec.layers_out &&
           !(spec.flags & CG_KEEP_ALL_LAYERS) && spec.max_layers <= (int)0x7fffffff;
}

// ---------------------------------------------------------------------------
// WgRunner
// ---------------------------------------------------------------------------
WgRunner::WgRunner(hipStream_t s) : stream_(s) {
    for (DevBuf *b : {&jobs_, &gsel_, &sizes_, &outs_, &ws_, &ticket_}) b->stream = s;
}

WgRunner::~WgRunner() {
    if (exec_) (void)hipGraphExecDestroy(exec_);
    if (graph_) (void)hipGraphDestroy(graph_);
    (void)hipStreamSynchronize(stream_);
    for (DevBuf *b : {&jobs_, &gsel_, &sizes_, &outs_, &ws_, &ticket_}) b->release();
}

namespace {

// Host tables of one small-job launch, jobs in launch order.
struct WgTables {
    std::vector<uint32_t> order;  // launch position -> item index
    std::vector<WgJobDev> jobs;
    std::vector<GenSel> gsel;
    uint64_t sizes_total = 0;     // layer-size entries of all jobs
    uint64_t slot_words = 0;      // words per bitmap of a device slot (0: no job needs one)
    uint32_t n_slot_jobs = 0;     // slot_first: jobs [0, n_slot_jobs) have n >= 9
    int n_max = 0;
};

// Largest jobs first (the queue then balances like longest-first); with
// slot_first the jobs whose bitmaps need a device slot come before all
// others. A job records at most min(max_layers, orbit) layer sizes: every
// recorded layer holds at least one state of the orbit.
WgTables wg_tables(const std::vector<WgItem> &items, bool slot_first) {
    const uint32_t nj = (uint32_t)items.size();
    WgTables T;
    T.order.resize(nj);
    for (uint32_t i = 0; i < nj; ++i) T.order[i] = i;
    std::stable_sort(T.order.begin(), T.order.end(), [&](uint32_t a, uint32_t b) {
        const JobSpec &x = *items[a].spec, &y = *items[b].spec;
        if (slot_first && (x.n > (int)kWgLdsN) != (y.n > (int)kWgLdsN)) return x.n > (int)kWgLdsN;
        const double cx = (double)factorial(x.n) * (x.k + 1), cy = (double)factorial(y.n) * (y.k + 1);
        return cx > cy;
    });
    T.jobs.resize(nj);
    for (uint32_t i = 0; i < nj; ++i) {
        const JobSpec &s = *items[T.order[i]].spec;
        if (!wg_eligible(s)) throw Error(CG_E_INVAL, "job not eligible for the small-job engine");
        WgJobDev &d = T.jobs[i];
        d.n = (uint32_t)s.n;
        d.k = (uint32_t)s.k;
        d.goff = (uint32_t)T.gsel.size();
        uint64_t key = 0;
        for (int q = 0; q < s.n; ++q) key |= (uint64_t)s.start[q] << (4 * (s.n - 1 - q));
        d.start_rank = (uint32_t)host_rank64(key, s.n);
        d.max_layers = (uint32_t)s.max_layers;
        d.pad = 0;
        d.max_frontier = s.max_frontier;
        d.sizes_off = T.sizes_total;
        T.sizes_total += std::min<uint64_t>((uint64_t)s.max_layers, factorial(s.n));
        for (int g = 0; g < s.k; ++g) T.gsel.push_back(make_gensel(s.n, s.gens.data() + (size_t)g * s.n));
        if (s.n > (int)kWgLdsN) {
            T.slot_words = std::max<uint64_t>(T.slot_words, (factorial(s.n) + 31) / 32);
            if (slot_first) T.n_slot_jobs = i + 1;
        }
        T.n_max = std::max(T.n_max, s.n);
    }
    if (T.gsel.empty()) T.gsel.push_back(GenSel{});
    T.slot_words = (T.slot_words + 63) / 64 * 64;
    return T;
}

// Copies the launch's outcomes into the callers' results.
void wg_results(std::vector<WgItem> &items, const WgTables &T, const uint64_t *hsz, const WgOutDev *ho, double ms,
                double t_submit, double t_admit, double t_done) {
    for (uint32_t i = 0; i < (uint32_t)T.jobs.size(); ++i) {
        const JobSpec &s = *items[T.order[i]].spec;
        cg_result_t *r = items[T.order[i]].res;
        const WgOutDev &o = ho[i];
        std::memset(r->layer_sizes, 0, sizeof(uint64_t) * (size_t)s.max_layers);
        const int nl = std::max(0, std::min(o.num_layers, s.max_layers));
        std::memcpy(r->layer_sizes, hsz + T.jobs[i].sizes_off, sizeof(uint64_t) * (size_t)nl);
        r->status = o.status;
        r->num_layers = nl;
        r->states_expanded = o.expanded;
        r->candidates = o.expanded * (uint64_t)s.k;
        r->device_ms = ms;
        r->n_kstats = 0;
        r->t_submit = t_submit;
        r->t_admit = t_admit;
        r->t_done = t_done;
    }
}

}  // namespace

// Workgroups of a launch: every job its own, at most as many as are
// resident at once.
static uint32_t wg_grid(uint32_t n_jobs, int block) {
    int occ = 0;
    CG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, wg_growth_kernel, block, 0));
    if (occ < 1) occ = 1;
    return (uint32_t)std::min<uint64_t>(n_jobs, (uint64_t)device_cus() * (uint64_t)occ);
}

uint64_t WgRunner::launch_bytes(const std::vector<WgItem> &items, const WgTuning &t) {
    if (items.empty()) return 0;
    const WgTables T = wg_tables(items, true);
    const uint32_t nj = (uint32_t)items.size();
    const uint64_t slots = T.slot_words ? std::min<uint64_t>(wg_grid(nj, t.block), T.n_slot_jobs) : 0;
    // every buffer as DevBuf rounds it (64 KiB) with its growth slack
    auto r = [](uint64_t b) { return ((uint64_t)(1.5 * (double)b) + (64u << 10) - 1) / (64u << 10) * (64u << 10); };
    return r(sizeof(WgJobDev) * nj) + r(sizeof(GenSel) * T.gsel.size()) + r(sizeof(uint64_t) * T.sizes_total) +
           r(sizeof(WgOutDev) * nj) + r(256) + r(slots * 3 * T.slot_words * sizeof(uint32_t));
}

uint64_t WgRunner::device_bytes() const {
    return jobs_.bytes + gsel_.bytes + sizes_.bytes + outs_.bytes + ws_.bytes + ticket_.bytes;
}

void WgRunner::release() {
    if (exec_) (void)hipGraphExecDestroy(exec_);
    if (graph_) (void)hipGraphDestroy(graph_);
    exec_ = nullptr;
    graph_ = nullptr;
    graph_key_.clear();
    for (DevBuf *b : {&jobs_, &gsel_, &sizes_, &outs_, &ws_, &ticket_}) b->release();
}

double WgRunner::run(std::vector<WgItem> &items, const WgTuning &t, double t_submit) {
    const uint32_t nj = (uint32_t)items.size();
    if (!nj) return 0.0;
    if (t.block < 64 || t.block > kWgMaxBlock || t.block % kWave) throw Error(CG_E_INVAL, "bad workgroup size");
    // jobs that need a device slot first: only as many workgroups as there
    // are such jobs own one
    const WgTables T = wg_tables(items, true);
    const uint64_t sizes_total = T.sizes_total, slot_words = T.slot_words;
    const uint32_t grid = wg_grid(nj, t.block);
    const uint32_t n_slot_jobs = T.n_slot_jobs;
    const uint32_t n_slot_blocks = slot_words ? std::min(grid, n_slot_jobs) : 0u;

    jobs_.ensure(sizeof(WgJobDev) * nj, 1.25);
    gsel_.ensure(sizeof(GenSel) * T.gsel.size(), 1.25);
    sizes_.ensure(sizeof(uint64_t) * sizes_total, 1.25);
    outs_.ensure(sizeof(WgOutDev) * nj, 1.25);
    ticket_.ensure(256);
    if (slot_words) ws_.ensure((size_t)n_slot_blocks * 3 * slot_words * sizeof(uint32_t));
    CG_HIP(hipMemcpyAsync(jobs_.p, T.jobs.data(), sizeof(WgJobDev) * nj, hipMemcpyHostToDevice, stream_));
    CG_HIP(hipMemcpyAsync(gsel_.p, T.gsel.data(), sizeof(GenSel) * T.gsel.size(), hipMemcpyHostToDevice, stream_));

    uint32_t *gbits = slot_words ? ws_.as<uint32_t>() : nullptr;
    const std::vector<uint64_t> key = {(uint64_t)(uintptr_t)jobs_.p, nj, (uint64_t)(uintptr_t)gsel_.p,
                                       (uint64_t)(uintptr_t)sizes_.p, (uint64_t)(uintptr_t)outs_.p,
                                       (uint64_t)(uintptr_t)ticket_.p, (uint64_t)(uintptr_t)gbits, slot_words,
                                       grid, (uint64_t)t.block};
    auto enqueue = [&]() {
        hipLaunchKernelGGL(clear_u32_kernel, dim3(1), dim3(64), 0, stream_, ticket_.as<uint32_t>(), 2u);
        hipLaunchKernelGGL(wg_growth_kernel, dim3(grid), dim3(t.block), 0, stream_, jobs_.as<const WgJobDev>(), nj,
                           n_slot_jobs, n_slot_blocks, gsel_.as<const GenSel>(), sizes_.as<uint64_t>(),
                           outs_.as<WgOutDev>(), ticket_.as<uint32_t>(), gbits, slot_words);
    };
    if (key != graph_key_) {
        // the graph is built node by node (no stream capture): a queue
        // reset followed by the persistent kernel
        if (exec_) (void)hipGraphExecDestroy(exec_);
        if (graph_) (void)hipGraphDestroy(graph_);
        exec_ = nullptr;
        graph_ = nullptr;
        graph_key_.clear();
        uint32_t *tk = ticket_.as<uint32_t>();
        uint32_t two = 2;
        void *clear_args[] = {&tk, &two};
        const WgJobDev *a_jobs = jobs_.as<const WgJobDev>();
        uint32_t a_nj = nj, a_slot_jobs = n_slot_jobs, a_slot_blocks = n_slot_blocks;
        const GenSel *a_gsel = gsel_.as<const GenSel>();
        uint64_t *a_sizes = sizes_.as<uint64_t>();
        WgOutDev *a_outs = outs_.as<WgOutDev>();
        uint32_t *a_gbits = gbits;
        uint64_t a_slot = slot_words;
        void *wg_args[] = {&a_jobs, &a_nj, &a_slot_jobs, &a_slot_blocks, &a_gsel, &a_sizes, &a_outs, &tk, &a_gbits,
                           &a_slot};
        hipKernelNodeParams p0{}, p1{};
        p0.func = reinterpret_cast<void *>(clear_u32_kernel);
        p0.gridDim = dim3(1);
        p0.blockDim = dim3(64);
        p0.sharedMemBytes = 0;
        p0.kernelParams = clear_args;
        p0.extra = nullptr;
        p1.func = reinterpret_cast<void *>(wg_growth_kernel);
        p1.gridDim = dim3(grid);
        p1.blockDim = dim3(t.block);
        p1.sharedMemBytes = 0;
        p1.kernelParams = wg_args;
        p1.extra = nullptr;
        hipGraphNode_t n0 = nullptr, n1 = nullptr;
        bool ok = hipGraphCreate(&graph_, 0) == hipSuccess;
        ok = ok && hipGraphAddKernelNode(&n0, graph_, nullptr, 0, &p0) == hipSuccess;
        ok = ok && hipGraphAddKernelNode(&n1, graph_, &n0, 1, &p1) == hipSuccess;
        ok = ok && hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0) == hipSuccess;
        if (ok) {
            graph_key_ = key;
            ++graph_captures_;
        } else {
            (void)hipGetLastError();
            if (exec_) (void)hipGraphExecDestroy(exec_);
            if (graph_) (void)hipGraphDestroy(graph_);
            exec_ = nullptr;
            graph_ = nullptr;
        }
    }
    hipEvent_t e0, e1;
    CG_HIP(hipEventCreate(&e0));
    CG_HIP(hipEventCreate(&e1));
    const double t_admit = now_seconds();
    CG_HIP(hipEventRecord(e0, stream_));
    if (exec_) {
        CG_HIP(hipGraphLaunch(exec_, stream_));
        ++graph_launches_;
    } else {
        enqueue();
        CG_HIP(hipGetLastError());
    }
    CG_HIP(hipEventRecord(e1, stream_));
    std::vector<uint64_t> hsz(sizes_total);
    std::vector<WgOutDev> ho(nj);
    CG_HIP(hipMemcpyAsync(hsz.data(), sizes_.p, sizeof(uint64_t) * sizes_total, hipMemcpyDeviceToHost, stream_));
    CG_HIP(hipMemcpyAsync(ho.data(), outs_.p, sizeof(WgOutDev) * nj, hipMemcpyDeviceToHost, stream_));
    CG_HIP(hipStreamSynchronize(stream_));
    float ms = 0;
    CG_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const double t_done = now_seconds();
    wg_results(items, T, hsz.data(), ho.data(), ms, t_submit, t_admit, t_done);
    return ms;
}

WgTuning tune_wg(std::vector<WgItem> &sample, WgRunner &r, double *best_ms_out) {
    WgTuning best;
    double best_ms = -1;
    for (int block : {256, 512, 1024}) {
        WgTuning t;
        t.block = block;
        r.run(sample, t, now_seconds());  // first run: graph build, warm caches
        const double ms = r.run(sample, t, now_seconds());
        if (best_ms < 0 || ms < best_ms) {
            best_ms = ms;
            best = t;
        }
    }
    if (best_ms_out) *best_ms_out = best_ms;
    return best;
}

// ---------------------------------------------------------------------------
// Small-job batches without allocation (cg_growth_batch_noalloc)
// ---------------------------------------------------------------------------
namespace {

constexpr size_t na_align(size_t x) { return (x + 255) & ~(size_t)255; }
// layout of the scratch array
constexpr size_t kNaOffTicket = 0;  // two uint32 queue tickets
constexpr size_t kNaOffOuts = 256;
constexpr size_t kNaOffJobs = na_align(kNaOffOuts + sizeof(WgOutDev) * kNoAllocMaxJobs);
constexpr size_t kNaOffGsel = na_align(kNaOffJobs + sizeof(WgJobDev) * kNoAllocMaxJobs);
constexpr size_t kNaOffSizes = na_align(kNaOffGsel + sizeof(GenSel) * kNoAllocMaxGens);
constexpr size_t kNaOffSlots = na_align(kNaOffSizes + sizeof(uint64_t) * kNoAllocMaxSizes);
// one n = 10 slot: three bitmaps of 10!/32 words, rounded up to 64 words
constexpr size_t kNaSlot10 = 3 * (((factorial(10) + 31) / 32 + 63) / 64 * 64) * sizeof(uint32_t);
static_assert(kNaOffSlots + 16 * kNaSlot10 <= kNoAllocScratchBytes, "room for at least 16 slots of n = 10");

constexpr int kNaMaxDevices = 64;
struct NaDevice {
    std::once_flag once;
    hipError_t err = hipSuccess;
    void *ptr = nullptr;  // the device's address of `scratch`
    std::mutex mu;        // one call at a time per device in this process
};
NaDevice g_na[kNaMaxDevices];

}  // namespace

void *noalloc_scratch(int dev) {
    if (dev < 0 || dev >= kNaMaxDevices) throw Error(CG_E_DEVICE, "device index beyond the no-allocation table");
    NaDevice &d = g_na[dev];
    // once per device, with that device current (the caller's): each GPU
    // holds its own copy of the array at its own address
    std::call_once(d.once, [&] { d.err = hipGetSymbolAddress(&d.ptr, HIP_SYMBOL(scratch)); });
    if (d.err != hipSuccess || !d.ptr)
        throw Error(CG_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(d.err));
    return d.ptr;
}

void run_batch_noalloc(int n_jobs, const cg_job_t *jobs, cg_result_t *results, hipStream_t stream) {
    const double t0 = now_seconds();
    if (n_jobs < 0 || n_jobs > (int)kNoAllocMaxJobs)
        throw Error(CG_E_INVAL, "cg_growth_batch_noalloc takes at most 4096 jobs");
    std::vector<JobSpec> specs;
    specs.reserve((size_t)n_jobs);
    std::vector<WgItem> items;
    std::vector<int> idx;
    for (int i = 0; i < n_jobs; ++i) {
        cg_result_t *r = &results[i];
        if (!r->layer_sizes) {
            r->status = CG_E_INVAL;
            r->num_layers = 0;
            continue;
        }
        try {
            specs.push_back(canonicalize(jobs[i], true));
        } catch (const Error &e) {
            r->status = e.code;
            r->num_layers = 0;
            continue;
        }
        if (!wg_eligible(specs.back())) {
            char buf[160];
            std::snprintf(buf, sizeof buf,
                          "job %d: cg_growth_batch_noalloc needs n <= 10, a permutation start and at most 128 "
                          "generators",
                          i);
            throw Error(CG_E_INVAL, buf);
        }
        idx.push_back(i);
    }
    for (size_t j = 0; j < specs.size(); ++j) items.push_back({&specs[j], &results[idx[j]]});
    if (items.empty()) return;
    const WgTables T = wg_tables(items, true);
    if (T.gsel.size() > kNoAllocMaxGens)
        throw Error(CG_E_INVAL, "cg_growth_batch_noalloc takes at most 32768 distinct generators in all");
    if (T.sizes_total > kNoAllocMaxSizes)
        throw Error(CG_E_INVAL, "cg_growth_batch_noalloc records at most 2^21 layer sizes in all "
                                "(sum over jobs of min(max_layers, n!))");
    const uint32_t nj = (uint32_t)items.size();
    int dev = 0;
    CG_HIP(hipGetDevice(&dev));
    unsigned char *base = static_cast<unsigned char *>(noalloc_scratch(dev));
    std::lock_guard<std::mutex> lk(g_na[dev].mu);

    uint32_t *ticket = reinterpret_cast<uint32_t *>(base + kNaOffTicket);
    WgOutDev *outs = reinterpret_cast<WgOutDev *>(base + kNaOffOuts);
    WgJobDev *djobs = reinterpret_cast<WgJobDev *>(base + kNaOffJobs);
    GenSel *dgsel = reinterpret_cast<GenSel *>(base + kNaOffGsel);
    uint64_t *dsizes = reinterpret_cast<uint64_t *>(base + kNaOffSizes);
    uint32_t *gbits = T.slot_words ? reinterpret_cast<uint32_t *>(base + kNaOffSlots) : nullptr;

    // the launch shape of cg_growth_batch for the batch's largest n
    const int block = T.n_max >= 10 ? 1024 : (T.n_max == 9 ? 512 : 256);
    const uint32_t grid = wg_grid(nj, block);
    // workgroups that own a slot: as many as the slot area holds, at most
    // one per job that needs one
    uint32_t n_slot_blocks = 0;
    if (gbits) {
        const uint64_t slot_bytes = 3 * T.slot_words * sizeof(uint32_t);
        const uint64_t fit = (kNoAllocScratchBytes - kNaOffSlots) / slot_bytes;
        n_slot_blocks = (uint32_t)std::min<uint64_t>({fit, (uint64_t)grid, (uint64_t)T.n_slot_jobs});
        if (n_slot_blocks < 1 || kNaOffSlots + (uint64_t)n_slot_blocks * slot_bytes > kNoAllocScratchBytes)
            throw Error(CG_E_DEVICE, "no-allocation slot layout");
    }
    CG_HIP(hipMemcpyAsync(djobs, T.jobs.data(), sizeof(WgJobDev) * nj, hipMemcpyHostToDevice, stream));
    CG_HIP(hipMemcpyAsync(dgsel, T.gsel.data(), sizeof(GenSel) * T.gsel.size(), hipMemcpyHostToDevice, stream));
    // the array keeps the last call's contents: the tickets start at zero
    hipLaunchKernelGGL(clear_u32_kernel, dim3(1), dim3(64), 0, stream, ticket, 2u);
    CG_HIP(hipGetLastError());
    const double t_admit = now_seconds();
    hipLaunchKernelGGL(wg_growth_kernel, dim3(grid), dim3(block), 0, stream, (const WgJobDev *)djobs, nj,
                       T.n_slot_jobs, n_slot_blocks, (const GenSel *)dgsel, dsizes, outs, ticket, gbits,
                       T.slot_words);
    CG_HIP(hipGetLastError());
    std::vector<uint64_t> hsz(T.sizes_total);
    std::vector<WgOutDev> ho(nj);
    CG_HIP(hipMemcpyAsync(hsz.data(), dsizes, sizeof(uint64_t) * T.sizes_total, hipMemcpyDeviceToHost, stream));
    CG_HIP(hipMemcpyAsync(ho.data(), outs, sizeof(WgOutDev) * nj, hipMemcpyDeviceToHost, stream));
    CG_HIP(hipStreamSynchronize(stream));
    const double t_done = now_seconds();
    // no events (they would be allocated): device_ms is the host-timed span
    // from the launch to the end of the read-back
    wg_results(items, T, hsz.data(), ho.data(), 1e3 * (t_done - t_admit), t0, t_admit, t_done);
}

// ---------------------------------------------------------------------------
// Bitmask engine host loop
// ---------------------------------------------------------------------------
std::string bitmask_unsupported(const JobSpec &spec) {
    if (spec.n > kBitmaskMaxN) return "the bitmask engine covers n <= 14";
    if (!start_is_permutation(spec)) return "the bitmask engine needs a start state that is a permutation";
    if (spec.k > kBitmapMaxK) return "the bitmask engine takes at most 128 generators";
    if (spec.layers_out || (spec.flags & CG_KEEP_ALL_LAYERS)) return "the bitmask engine does not export layers";
    return "";
}

void run_bitmask(const JobSpec &spec, cg_result_t *res, hipStream_t s) {
    const std::string why = bitmask_unsupported(spec);
    if (!why.empty()) throw Error(CG_E_INVAL, why);
    const double t0 = now_seconds();
    const int n = spec.n, k = spec.k;
    uint64_t *sizes = res->layer_sizes;
    std::memset(sizes, 0, sizeof(uint64_t) * (size_t)spec.max_layers);
    sizes[0] = 1;
    res->status = CG_OK;
    res->num_layers = 1;
    res->states_expanded = 0;
    res->candidates = 0;
    res->n_kstats = 0;

    const uint64_t S = factorial(n);
    const uint64_t W = (S + 31) / 32;
    const uint64_t nchunks = (W + kChunkWords - 1) / kChunkWords;
    const uint64_t sw = (nchunks + 31) / 32;
    DevBuf vis, cur, nxt, scur, snxt, gsel, cnt;
    for (DevBuf *b : {&vis, &cur, &nxt, &scur, &snxt, &gsel, &cnt}) b->stream = s;
    vis.ensure(W * 4);
    cur.ensure(W * 4);
    nxt.ensure(W * 4);
    scur.ensure(sw * 4);
    snxt.ensure(sw * 4);
    cnt.ensure(64);
    std::vector<GenSel> hs(std::max(1, k));
    for (int g = 0; g < k; ++g) hs[g] = make_gensel(n, spec.gens.data() + (size_t)g * n);
    gsel.ensure(sizeof(GenSel) * hs.size());
    CG_HIP(hipMemcpyAsync(gsel.p, hs.data(), sizeof(GenSel) * hs.size(), hipMemcpyHostToDevice, s));
    CG_HIP(hipMemsetAsync(vis.p, 0, W * 4, s));
    CG_HIP(hipMemsetAsync(cur.p, 0, W * 4, s));
    CG_HIP(hipMemsetAsync(nxt.p, 0, W * 4, s));
    CG_HIP(hipMemsetAsync(scur.p, 0, sw * 4, s));
    CG_HIP(hipMemsetAsync(snxt.p, 0, sw * 4, s));
    uint64_t key0 = 0;
    for (int q = 0; q < n; ++q) key0 |= (uint64_t)spec.start[q] << (4 * (n - 1 - q));
    hipLaunchKernelGGL(bm_seed_kernel, dim3(1), dim3(1), 0, s, vis.as<uint32_t>(), cur.as<uint32_t>(),
                       scur.as<uint32_t>(), host_rank64(key0, n), cnt.as<unsigned long long>());
    CG_HIP(hipGetLastError());

    hipEvent_t e0, e1;
    CG_HIP(hipEventCreate(&e0));
    CG_HIP(hipEventCreate(&e1));
    CG_HIP(hipEventRecord(e0, s));
    const uint32_t grid = (uint32_t)std::min<uint64_t>(nchunks, (uint64_t)device_cus() * 16);
    uint64_t *host_cnt = nullptr;
    CG_HIP(hipHostMalloc((void **)&host_cnt, sizeof(uint64_t), hipHostMallocDefault));
    uint32_t *pc = cur.as<uint32_t>(), *pn = nxt.as<uint32_t>(), *sc = scur.as<uint32_t>(),
             *sn = snxt.as<uint32_t>();
    uint64_t F = 1;
    int layers = 1, status = CG_OK;
    try {
        for (;;) {
            if (k == 0) break;
            if (spec.max_frontier && F > spec.max_frontier) {
                status = CG_TRUNCATED;
                break;
            }
            if (layers >= spec.max_layers) {
                status = CG_TRUNCATED;
                break;
            }
            with_bm_n(n, [&](auto NN) {
                hipLaunchKernelGGL(bm_expand_kernel<decltype(NN)::value>, dim3(grid), dim3(kBmBlock), 0, s, pc, sc,
                                   vis.as<const uint32_t>(), pn, sn, W, nchunks, gsel.as<const GenSel>(), k);
            });
            CG_HIP(hipGetLastError());
            hipLaunchKernelGGL(bm_fold_kernel, dim3(grid), dim3(kBmBlock), 0, s, vis.as<uint32_t>(), pc, sc, pn, sn,
                               W, nchunks, cnt.as<unsigned long long>());
            CG_HIP(hipGetLastError());
            // the expanded layer's summary becomes the next layer's: clear it
            hipLaunchKernelGGL(bm_clear_kernel, dim3((uint32_t)std::min<uint64_t>((sw + 255) / 256, 4096)),
                               dim3(256), 0, s, sc, sw, (unsigned long long *)nullptr);
            CG_HIP(hipGetLastError());
            CG_HIP(hipMemcpyAsync(host_cnt, cnt.p, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
            hipLaunchKernelGGL(bm_clear_kernel, dim3(1), dim3(64), 0, s, (uint32_t *)nullptr, 0ull,
                               cnt.as<unsigned long long>());
            CG_HIP(hipStreamSynchronize(s));
            const uint64_t N = *host_cnt;
            res->states_expanded += F;
            res->candidates += F * (uint64_t)k;
            std::swap(pc, pn);
            std::swap(sc, sn);
            if (N == 0) break;
            sizes[layers++] = N;
            F = N;
        }
    } catch (...) {
        (void)hipStreamSynchronize(s);
        (void)hipHostFree(host_cnt);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    CG_HIP(hipEventRecord(e1, s));
    CG_HIP(hipEventSynchronize(e1));
    float ms = 0;
    CG_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipHostFree(host_cnt);
    for (DevBuf *b : {&vis, &cur, &nxt, &scur, &snxt, &gsel, &cnt}) b->release();
    res->device_ms = ms;
    res->status = status;
    res->num_layers = layers;
    res->t_submit = t0;
    res->t_admit = t0;
    res->t_done = now_seconds();
}

}  // namespace cg
