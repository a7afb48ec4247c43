// Unique + set difference + stream compaction of one layer's sorted
// candidates.
//
// A candidate is a new state of layer d+1 iff it is the first of its run of
// equal keys and it belongs neither to layer d nor to layer d-1. For a
// generating set closed under inverses (the standard undirected case of the
// section "Largest diameters found (and known) for n <= 15") every
// neighbour of a state at distance d is at distance d-1, d or d+1 (distance
// as defined in section "Reminder on Cayley graphs, diameters, growth"), so
// these two layers are the only earlier states a candidate can hit.
//
// One 4096-key tile per block:
//   * keys load coalesced into LDS; thread t takes keys 16t..16t+15 (a
//     padded layout keeps these reads free of bank conflicts);
//   * wave 0 locates the tile's key range in each reference layer with
//     64-way ballot searches; the matching slice is streamed through LDS
//     in chunks and every thread merges its 16 sorted keys against it with
//     a galloping search;
//   * survivors are counted, block-scanned, offset by a decoupled look-back
//     over the tiles before, staged in LDS and written out contiguously, so
//     the new layer comes out sorted.
#include "internal.h"
#include "device_util.h"

namespace cg {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
constexpr int kIpt = 16;
constexpr int kTile = kBlock * kIpt;  // 4096
constexpr int kRef = 2048;            // reference keys per LDS chunk

__device__ __forceinline__ uint32_t pad(uint32_t i) { return i + (i >> 4); }

// First index in [pos, m) of the sorted LDS array `a` with a[idx] >= key,
// or m; galloping from pos.
__device__ __forceinline__ uint32_t gallop_lb(const uint64_t *a, uint32_t pos, uint32_t m,
                                              uint64_t key) {
    if (pos >= m || a[pos] >= key) return pos;
    uint32_t lo = pos, step = 1, hi = m;  // a[lo] < key
    for (;;) {
        const uint32_t probe = lo + step;
        if (probe >= m) break;
        if (a[probe] >= key) {
            hi = probe;
            break;
        }
        lo = probe;
        step <<= 1;
    }
    uint32_t L = lo + 1, H = hi;  // answer in [L, H]
    while (L < H) {
        const uint32_t mid = (L + H) >> 1;
        if (a[mid] < key)
            L = mid + 1;
        else
            H = mid;
    }
    return L;
}

__global__ __launch_bounds__(kBlock) void dedup_kernel(
    const uint64_t *__restrict__ S, uint64_t C, const uint64_t *__restrict__ A, uint64_t na,
    const uint64_t *__restrict__ B, uint64_t nb, uint64_t *__restrict__ out, uint64_t out_cap,
    uint64_t *__restrict__ out_count, uint64_t *__restrict__ status,
    uint32_t *__restrict__ ticket, uint32_t epoch, uint32_t ntiles, uint32_t *__restrict__ err) {
    __shared__ uint64_t s_keys[kTile + kTile / 16];
    __shared__ uint64_t s_ref[kRef];
    __shared__ uint64_t s_bounds[2];
    __shared__ uint32_t s_scan[kWaves];
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_off;

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wave = tid / kWave;

    if (tid == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint64_t base = (uint64_t)tile * kTile;
    const uint64_t left = C - base;
    const uint32_t nvalid = (uint32_t)(left < (uint64_t)kTile ? left : (uint64_t)kTile);

#pragma unroll
    for (int j = 0; j < kIpt; ++j) {
        const uint32_t i = j * kBlock + tid;
        s_keys[pad(i)] = i < nvalid ? S[base + i] : kSentinel;
    }
    const bool has_prev = base > 0;
    const uint64_t prev_global = has_prev ? S[base - 1] : 0;
    __syncthreads();

    uint64_t k[kIpt];
    uint32_t keep = 0;
#pragma unroll
    for (int j = 0; j < kIpt; ++j) {
        const uint32_t idx = tid * kIpt + j;
        k[j] = s_keys[pad(idx)];
        uint64_t prev;
        bool first;
        if (j > 0) {
            prev = k[j - 1];
            first = false;
        } else if (tid > 0) {
            prev = s_keys[pad(idx - 1)];
            first = false;
        } else {
            prev = prev_global;
            first = !has_prev;
        }
        if (idx < nvalid && (first || k[j] != prev)) keep |= 1u << j;
    }
    const uint64_t kfirst = s_keys[pad(0)];
    const uint64_t klast = s_keys[pad(nvalid - 1)];

    for (int r = 0; r < 2; ++r) {
        const uint64_t *R = r == 0 ? A : B;
        const uint64_t nr = r == 0 ? na : nb;
        if (nr == 0) continue;
        if (wave == 0) {
            const uint64_t lo = wave_search(R, nr, kfirst, false);
            const uint64_t hi = wave_search(R, nr, klast, true);
            if (lane == 0) {
                s_bounds[0] = lo;
                s_bounds[1] = hi;
            }
        }
        __syncthreads();
        const uint64_t lo = s_bounds[0], hi = s_bounds[1];
        __syncthreads();
        for (uint64_t c0 = lo; c0 < hi; c0 += kRef) {
            const uint64_t rem = hi - c0;
            const uint32_t m = (uint32_t)(rem < (uint64_t)kRef ? rem : (uint64_t)kRef);
            for (uint32_t i = tid; i < m; i += kBlock) s_ref[i] = R[c0 + i];
            __syncthreads();
            if (keep) {
                uint32_t pos = 0;
#pragma unroll
                for (int j = 0; j < kIpt; ++j) {
                    if ((keep >> j) & 1u) {
                        pos = gallop_lb(s_ref, pos, m, k[j]);
                        if (pos < m && s_ref[pos] == k[j]) keep &= ~(1u << j);
                    }
                }
            }
            __syncthreads();
        }
    }

    // compaction
    const uint32_t cnt = (uint32_t)__popc(keep);
    uint32_t total;
    const uint32_t toff = block_excl_scan<kWaves>(cnt, s_scan, &total);
    if (tid == 0) {
        uint64_t *my = status + tile;
        uint64_t excl = 0;
        if (tile == 0) {
            lb_store(my, lb_word(epoch, kFlagInclusive, total));
        } else {
            lb_store(my, lb_word(epoch, kFlagAggregate, total));
            excl = lb_lookback(status, 1, tile, epoch, err);
            lb_store(my, lb_word(epoch, kFlagInclusive, excl + total));
        }
        s_off = excl;
        if (tile == ntiles - 1) *out_count = excl + total;
    }
    {
        uint32_t r = toff;
#pragma unroll
        for (int j = 0; j < kIpt; ++j)
            if ((keep >> j) & 1u) s_keys[pad(r++)] = k[j];
    }
    __syncthreads();
    const uint64_t off = s_off;
    for (uint32_t i = tid; i < total; i += kBlock) {
        if (off + i < out_cap)
            out[off + i] = s_keys[pad(i)];
        else
            atomicOr(err, 4u);  // more survivors than the output holds
    }
}

}  // namespace

uint64_t dedup_status_words(uint64_t C) { return (C + kTile - 1) / kTile; }

void launch_dedup(const uint64_t *sorted, uint64_t C, const uint64_t *a, uint64_t na,
                  const uint64_t *b, uint64_t nb, uint64_t *out, uint64_t out_cap,
                  uint64_t *d_count, PipeWork &w) {
    uint32_t *ticket = w.tickets() + 31;
    // clears the ticket and the output count (a kernel, not a memset, so the
    // sequence stays valid inside a captured graph)
    launch_clear(ticket, 1, d_count, 1, w.stream);
    if (C == 0) return;
    const uint32_t ntiles = (uint32_t)dedup_status_words(C);
    w.ensure_status(ntiles);
    const uint32_t epoch = w.next_epoch();
    if (w.prof) w.prof->begin(K_DEDUP);
    hipLaunchKernelGGL(dedup_kernel, dim3(ntiles), dim3(kBlock), 0, w.stream, sorted, C, a, na, b, nb,
                       out, out_cap, d_count, w.status.as<uint64_t>(), ticket, epoch, ntiles, w.err());
    CG_HIP(hipGetLastError());
    // algorithmic traffic: candidates and both reference layers are read
    // once; the 8N bytes of the output are added by the caller once N is
    // known
    if (w.prof) w.prof->end(K_DEDUP, 8.0 * (double)(C + na + nb), (double)C);
}

}  // namespace cg
