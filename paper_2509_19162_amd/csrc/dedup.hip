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
//   * a separate small kernel first finds, for every tile, the slice of each
//     reference layer between the tile's first and last key (binary
//     searches, one thread each), so no tile waits on a search;
//   * every reference key of the slice (usually far fewer than the
//     candidates) looks itself up in the tile, sorted in LDS, with a
//     branchless binary search and marks the equal candidate; when a small
//     candidate array meets large reference layers the marking runs over
//     the whole reference layers instead, one thread per reference key;
//   * survivors are compacted within the tile and parked in a scratch
//     buffer with their count; no tile waits on another;
//   * a small scan turns the counts into offsets, and a gather moves each
//     tile's survivors to their final place, so the new layer comes out
//     sorted and contiguous.
#include <algorithm>

#include "internal.h"
#include "device_util.h"
#include "perm_rank.h"

namespace cg {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
#ifndef CG_DEDUP_IPT
#define CG_DEDUP_IPT 16
#endif
constexpr int kIpt = CG_DEDUP_IPT;
constexpr int kTile = kBlock * kIpt;  // 4096 candidates per dedup tile by default
#ifndef CG_GATHER_TILES
#define CG_GATHER_TILES 4
#endif
constexpr int kGatherTiles = CG_GATHER_TILES;  // dedup tiles per gather block
// reference keys per thread loaded with the tile and searched in lockstep:
// kRefIptFew, or kRefIptMany when the references average more than
// kRefManyAt per thread (about 32/k of them for k generators: S_16 LRX,
// k = 3, set difference and compaction 154 -> 142 ms with 8; with 11
// generators 4 is faster, 11.2 against 13.1 ms on S_12 pancake)
constexpr int kRefIptFew = 4;
constexpr int kRefIptMany = 8;
constexpr uint64_t kRefManyAt = 6;
#ifndef CG_DEDUP_LOCKSTEP
#define CG_DEDUP_LOCKSTEP 1  // the tile's first references searched in lockstep
#endif
// largest candidate array looked up from the reference side (4 MB of u32)
constexpr uint64_t kMarkMaxCandidates = 1u << 20;

__device__ __forceinline__ uint32_t pad(uint32_t i) { return i + (i >> 4); }

// Candidates are packed 64-bit keys, or (n <= 12) their 32-bit
// lexicographic ranks. The policy turns a layer key into the candidates'
// form and a candidate back into a layer key; both preserve order.
struct PackedKeys {
    using K = uint64_t;
    using Ref = uint64_t;  // reference layers as stored
    static constexpr bool kConvert = false;  // survivors are moved as they are
    int n;
    __device__ __forceinline__ K from_layer(uint64_t x) const { return x; }
    __device__ __forceinline__ uint64_t to_layer(K x) const { return x; }
};
template <int N>
struct RankedKeys {
    using K = uint32_t;
    using Ref = uint64_t;
    static constexpr bool kConvert = true;
    int n;
    __device__ __forceinline__ K from_layer(uint64_t x) const { return perm_rank_t<N>(x); }
    __device__ __forceinline__ uint64_t to_layer(K x) const { return perm_unrank_t<N>(x); }
};
// Reference layers given by their ranks (kept beside the packed layers):
// no ranking in the set difference.
template <int N>
struct RankedRefs {
    using K = uint32_t;
    using Ref = uint32_t;
    static constexpr bool kConvert = true;
    int n;
    __device__ __forceinline__ K from_layer(uint32_t x) const { return x; }
    __device__ __forceinline__ uint64_t to_layer(K x) const { return perm_unrank_t<N>(x); }
};
// Candidates as 64-bit ranks (n = 13..16); reference layers packed, or
// given by their 64-bit ranks (Ranked64Refs).
template <int N>
struct Ranked64Refs {
    using K = uint64_t;
    using Ref = uint64_t;
    static constexpr bool kConvert = true;
    int n;
    __device__ __forceinline__ K from_layer(uint64_t x) const { return x; }
    __device__ __forceinline__ uint64_t to_layer(K x) const { return perm_unrank_t<N, uint64_t>(x); }
};
template <int N>
struct Ranked64Keys {
    using K = uint64_t;
    using Ref = uint64_t;
    static constexpr bool kConvert = true;
    int n;
    __device__ __forceinline__ K from_layer(uint64_t x) const { return perm_rank_t<N, uint64_t>(x); }
    __device__ __forceinline__ uint64_t to_layer(K x) const { return perm_unrank_t<N, uint64_t>(x); }
};

// bounds[4t + 0/1]: lower bound of tile t's first key / upper bound of its
// last key in A; bounds[4t + 2/3]: the same in B. One thread per bound; the
// searches of neighbouring tiles share their upper levels in the caches.
template <class P>
__global__ __launch_bounds__(256) void tile_bounds_kernel(
    P pol, const typename P::K *__restrict__ S, uint64_t C, const typename P::Ref *__restrict__ A, uint64_t na,
    const typename P::Ref *__restrict__ B, uint64_t nb, uint64_t *__restrict__ bounds, uint32_t ntiles) {
    using K = typename P::K;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * ntiles) return;
    const uint32_t t = i >> 2, w = i & 3u;
    const typename P::Ref *R = w < 2 ? A : B;
    const uint64_t nr = w < 2 ? na : nb;
    const bool upper = (w & 1u) != 0;
    const uint64_t end = ((uint64_t)t + 1) * kTile < C ? ((uint64_t)t + 1) * kTile : C;
    const K key = upper ? S[end - 1] : S[(uint64_t)t * kTile];
    uint64_t lo = 0, hi = nr;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        const K v = pol.from_layer(R[mid]);
        if (upper ? (v <= key) : (v < key))
            lo = mid + 1;
        else
            hi = mid;
    }
    bounds[i] = lo;
}

// Phase 1: one tile per block (no inter-tile dependency): unique + set
// difference, survivors compacted within the tile into tmp[tile*kTile ..]
// and counted in cnt[tile].
// Reference-heavy layers (a small candidate array against large reference
// layers, as at the end of a search): each reference key is looked up in the
// whole sorted candidate array, which is small enough to stay in the caches,
// and the first equal candidate is flagged. With per-tile slices all those
// references would fall to the one or two blocks whose key range covers them.
template <class P>
__global__ __launch_bounds__(256) void mark_refs_kernel(P pol, const typename P::K *__restrict__ S, uint64_t C,
                                                        const typename P::Ref *__restrict__ R, uint64_t nr,
                                                        uint8_t *__restrict__ kill) {
    using K = typename P::K;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nr; i += stride) {
        const K key = pol.from_layer(R[i]);
        uint64_t lo = 0, hi = C;
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (S[mid] < key)
                lo = mid + 1;
            else
                hi = mid;
        }
        if (lo < C && S[lo] == key) kill[lo] = 1;
    }
}

template <class P, int kRefIpt>
__global__ __launch_bounds__(kBlock) void dedup_local_kernel(
    P pol, const typename P::K *__restrict__ S, uint64_t C, const typename P::Ref *__restrict__ A, uint64_t na,
    const typename P::Ref *__restrict__ B, uint64_t nb, const uint64_t *__restrict__ bounds,
    const uint8_t *__restrict__ gkill, typename P::K *__restrict__ tmp, uint32_t *__restrict__ cnt) {
    using K = typename P::K;
    __shared__ K s_keys[kTile + kTile / 16];
    __shared__ uint8_t s_kill[kTile];
    __shared__ uint32_t s_scan[kWaves];

    const uint32_t tid = threadIdx.x;
    const uint32_t tile = blockIdx.x;
    const uint64_t base = (uint64_t)tile * kTile;
    const uint64_t left = C - base;
    const uint32_t nvalid = (uint32_t)(left < (uint64_t)kTile ? left : (uint64_t)kTile);

    // The slices of the reference layers come first: the loads of the first
    // kRefIpt references per thread then go out together with the tile's
    // candidates instead of one latency after another.
    uint64_t bnd[4] = {0, 0, 0, 0};
    if (gkill) na = nb = 0;  // matches already flagged by mark_refs_kernel
    if (na) {
        bnd[0] = bounds[4 * (uint64_t)tile];
        bnd[1] = bounds[4 * (uint64_t)tile + 1];
    }
    if (nb) {
        bnd[2] = bounds[4 * (uint64_t)tile + 2];
        bnd[3] = bounds[4 * (uint64_t)tile + 3];
    }
    K kin[kIpt];
#pragma unroll
    for (int j = 0; j < kIpt; ++j) {
        const uint32_t i = j * kBlock + tid;
        kin[j] = i < nvalid ? S[base + i] : (K)kSentinel;
    }
    const bool has_prev = base > 0;
    const K prev_global = has_prev ? S[base - 1] : (K)0;
    // references of both slices as one list: A's slice, then B's
    const uint64_t n_a = bnd[1] - bnd[0];
    const uint64_t n_ref = n_a + (bnd[3] - bnd[2]);
    auto ref_at = [&](uint64_t t) -> K {
        return pol.from_layer(t < n_a ? A[bnd[0] + t] : B[bnd[2] + (t - n_a)]);
    };
    K ref[kRefIpt];
#pragma unroll
    for (int u = 0; u < kRefIpt; ++u) {
        const uint64_t t = (uint64_t)u * kBlock + tid;
        ref[u] = t < n_ref ? ref_at(t) : (K)0;
    }
#pragma unroll
    for (int j = 0; j < kIpt; ++j) {
        const uint32_t i = j * kBlock + tid;
        s_keys[pad(i)] = kin[j];
        s_kill[i] = (gkill && i < nvalid) ? gkill[base + i] : 0;
    }
    __syncthreads();

    // Reference keys in the tile's range are far fewer than candidates: each
    // one looks itself up in the sorted tile (12 LDS probes) and marks the
    // first equal candidate; later copies of a key are dropped as repeats.
    auto mark = [&](K key) {
        uint32_t pos = 0, len = nvalid;
        while (len > 1) {
            const uint32_t half = len >> 1;
            pos = s_keys[pad(pos + half)] < key ? pos + half : pos;
            len -= half;
        }
        const uint32_t lb = pos + (s_keys[pad(pos)] < key ? 1u : 0u);
        if (lb < nvalid && s_keys[pad(lb)] == key) s_kill[lb] = 1;
    };
#if CG_DEDUP_LOCKSTEP
    // The first kRefIpt references of each thread search together: the
    // tile is padded to kTile (a power of two) with all-ones keys, so a
    // fixed log2(kTile)-step lower bound over it needs no length and the
    // searches' LDS probes overlap instead of following one another.
    static_assert((kTile & (kTile - 1)) == 0, "tile length is a power of two");
    {
        uint32_t pos[kRefIpt];
#pragma unroll
        for (int u = 0; u < kRefIpt; ++u) pos[u] = 0;
#pragma unroll
        for (uint32_t step = kTile / 2; step >= 1; step >>= 1) {
#pragma unroll
            for (int u = 0; u < kRefIpt; ++u)
                pos[u] = s_keys[pad(pos[u] + step - 1)] < ref[u] ? pos[u] + step : pos[u];
        }
#pragma unroll
        for (int u = 0; u < kRefIpt; ++u) {
            const uint32_t lb = pos[u] + (s_keys[pad(pos[u])] < ref[u] ? 1u : 0u);
            if ((uint64_t)u * kBlock + tid < n_ref && lb < nvalid && s_keys[pad(lb)] == ref[u])
                s_kill[lb] = 1;
        }
    }
#else
#pragma unroll
    for (int u = 0; u < kRefIpt; ++u)
        if ((uint64_t)u * kBlock + tid < n_ref) mark(ref[u]);
#endif
    for (uint64_t t = (uint64_t)kRefIpt * kBlock + tid; t < n_ref; t += kBlock) mark(ref_at(t));
    __syncthreads();

    K k[kIpt];
    uint32_t keep = 0;
#pragma unroll
    for (int j = 0; j < kIpt; ++j) {
        const uint32_t idx = tid * kIpt + j;
        k[j] = s_keys[pad(idx)];
        K prev;
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
        if (idx < nvalid && (first || k[j] != prev) && !s_kill[idx]) keep |= 1u << j;
    }

    uint32_t total;
    const uint32_t toff = block_excl_scan<kWaves>((uint32_t)__popc(keep), s_scan, &total);
    {
        uint32_t r = toff;
#pragma unroll
        for (int j = 0; j < kIpt; ++j)
            if ((keep >> j) & 1u) s_keys[pad(r++)] = k[j];
    }
    __syncthreads();
    for (uint32_t i = tid; i < total; i += kBlock) tmp[base + i] = s_keys[pad(i)];
    if (tid == 0) cnt[tile] = total;
}

__global__ void fill_bytes_kernel(uint8_t *__restrict__ p, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Phase 2: exclusive prefix of the per-tile counts, 1024 tiles per block,
// blocks chained by a wave-parallel decoupled look-back (uniform work).
constexpr int kScanBlock = 256;
constexpr int kScanIpt = 4;
constexpr int kScanTile = kScanBlock * kScanIpt;

__global__ __launch_bounds__(kScanBlock) void count_scan_kernel(
    const uint32_t *__restrict__ cnt, uint32_t n, uint64_t *__restrict__ off,
    uint64_t *__restrict__ total_out, uint64_t *__restrict__ status, uint32_t *__restrict__ ticket,
    uint32_t epoch, uint32_t nblocks, uint32_t *__restrict__ err) {
    __shared__ uint64_t s_scan[kScanBlock / kWave];
    __shared__ uint32_t s_blk;
    __shared__ uint64_t s_prefix;
    const uint32_t tid = threadIdx.x;
    if (tid == 0) s_blk = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t blk = s_blk;
    const uint64_t first = (uint64_t)blk * kScanTile + (uint64_t)tid * kScanIpt;
    uint64_t v[kScanIpt];
    uint64_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanIpt; ++j) {
        v[j] = first + j < n ? cnt[first + j] : 0;
        sum += v[j];
    }
    uint64_t block_total;
    const uint64_t ex = block_excl_scan<kScanBlock / kWave>(sum, s_scan, &block_total);
    if (tid < kWave) {
        const uint32_t lane = lane_id();
        uint64_t prefix = 0;
        if (blk == 0) {
            if (lane == 0) lb_store(status + blk, lb_word(epoch, kFlagInclusive, block_total));
        } else {
            if (lane == 0) lb_store(status + blk, lb_word(epoch, kFlagAggregate, block_total));
            prefix = lb_lookback_wave(status, blk, epoch, err);
            if (lane == 0) lb_store(status + blk, lb_word(epoch, kFlagInclusive, prefix + block_total));
        }
        if (lane == 0) {
            s_prefix = prefix;
            if (blk == nblocks - 1) *total_out = prefix + block_total;
        }
    }
    __syncthreads();
    uint64_t run = s_prefix + ex;
#pragma unroll
    for (int j = 0; j < kScanIpt; ++j) {
        if (first + j < n) off[first + j] = run;
        run += v[j];
    }
}

// Phase 3: move each tile's survivors to their final place (and, for
// ranked candidates, their ranks to rank_out when it is given). For ranked
// candidates a block takes kGatherTiles consecutive tiles: a tile keeps a
// few hundred survivors in the large layers, each is unranked on the way,
// and one block per tile would spend most of its life waiting on its one
// load. In each round a thread first loads its survivor of every tile of
// the block, then converts and stores them. Packed survivors only move, and
// there one tile per block measured faster.
template <class P>
constexpr int gather_tiles() {
    return P::kConvert ? kGatherTiles : 1;
}

template <class P>
__global__ __launch_bounds__(kBlock) void gather_kernel(P pol, const typename P::K *__restrict__ tmp,
                                                        const uint32_t *__restrict__ cnt,
                                                        const uint64_t *__restrict__ off, uint32_t ntiles,
                                                        uint64_t *__restrict__ out, uint64_t out_cap,
                                                        typename P::K *__restrict__ rank_out,
                                                        uint32_t *__restrict__ err) {
    using K = typename P::K;
    constexpr int kT = gather_tiles<P>();
    const uint32_t t0 = blockIdx.x * (uint32_t)kT;
    const uint32_t tid = threadIdx.x;
    auto put = [&](uint64_t dst, K v) {
        if (dst < out_cap) {
            out[dst] = pol.to_layer(v);
            if constexpr (P::kConvert)
                if (rank_out) rank_out[dst] = v;
        } else {
            atomicOr(err, 4u);  // more survivors than the output holds
        }
    };
    uint32_t c[kT];
    uint64_t o[kT];
    uint32_t cmax = 0;
#pragma unroll
    for (int t = 0; t < kT; ++t) {
        const bool in = t0 + t < ntiles;
        c[t] = in ? cnt[t0 + t] : 0u;
        o[t] = in ? off[t0 + t] : 0ull;
        cmax = c[t] > cmax ? c[t] : cmax;
    }
    for (uint32_t i = tid; i < cmax; i += kBlock) {
        K v[kT];
#pragma unroll
        for (int t = 0; t < kT; ++t)
            if (i < c[t]) v[t] = tmp[(uint64_t)(t0 + t) * kTile + i];
#pragma unroll
        for (int t = 0; t < kT; ++t)
            if (i < c[t]) put(o[t] + i, v[t]);
    }
}

}  // namespace

uint64_t dedup_status_words(uint64_t C) {
    const uint64_t tiles = (C + kTile - 1) / kTile;
    return (tiles + kScanTile - 1) / kScanTile;
}

namespace {

template <class P>
void dedup_count_impl(P pol, const typename P::K *sorted, uint64_t C, const typename P::Ref *a, uint64_t na,
                      const typename P::Ref *b, uint64_t nb, typename P::K *tmp, uint64_t *d_count, PipeWork &w) {
    uint32_t *ticket = w.tickets() + 31;
    // clears the ticket and the output count (a kernel, not a memset, so the
    // sequence stays valid inside a captured graph)
    launch_clear(ticket, 1, d_count, 1, w.stream);
    w.dedup_tiles = 0;
    if (C == 0) return;
    const uint32_t ntiles = (uint32_t)((C + kTile - 1) / kTile);
    const uint32_t nscan = (ntiles + kScanTile - 1) / kScanTile;
    w.ensure_status(nscan);
    w.bounds.ensure((size_t)ntiles * 4 * sizeof(uint64_t), 1.25);
    w.tile_cnt.ensure((size_t)ntiles * sizeof(uint32_t), 1.25);
    w.tile_off.ensure((size_t)ntiles * sizeof(uint64_t), 1.25);
    const uint32_t epoch = w.next_epoch();
    if (w.prof) w.prof->begin(K_DEDUP);
    const bool ref_heavy = C <= kMarkMaxCandidates && na + nb > 4 * C;
    const uint8_t *gkill = nullptr;
    if (ref_heavy) {
        w.kill.ensure(C + 64, 1.25);
        hipLaunchKernelGGL(fill_bytes_kernel, dim3((uint32_t)((C + 255) / 256)), dim3(256), 0, w.stream,
                           w.kill.as<uint8_t>(), C);
        CG_HIP(hipGetLastError());
        auto blocks = [](uint64_t m) { return (uint32_t)std::min<uint64_t>((m + 255) / 256, 1u << 16); };
        if (na)
            hipLaunchKernelGGL(mark_refs_kernel<P>, dim3(blocks(na)), dim3(256), 0, w.stream, pol, sorted, C, a, na,
                               w.kill.as<uint8_t>());
        if (nb)
            hipLaunchKernelGGL(mark_refs_kernel<P>, dim3(blocks(nb)), dim3(256), 0, w.stream, pol, sorted, C, b, nb,
                               w.kill.as<uint8_t>());
        CG_HIP(hipGetLastError());
        gkill = w.kill.as<const uint8_t>();
    } else if (na || nb) {
        hipLaunchKernelGGL(tile_bounds_kernel<P>, dim3((4 * ntiles + 255) / 256), dim3(256), 0, w.stream,
                           pol, sorted, C, a, na, b, nb, w.bounds.as<uint64_t>(), ntiles);
        CG_HIP(hipGetLastError());
    }
    // references per thread of an average tile
    const bool many = !gkill && (na + nb) * (uint64_t)kTile > kRefManyAt * kBlock * C;
    if (many)
        hipLaunchKernelGGL((dedup_local_kernel<P, kRefIptMany>), dim3(ntiles), dim3(kBlock), 0, w.stream, pol, sorted,
                           C, a, na, b, nb, w.bounds.as<const uint64_t>(), gkill, tmp, w.tile_cnt.as<uint32_t>());
    else
        hipLaunchKernelGGL((dedup_local_kernel<P, kRefIptFew>), dim3(ntiles), dim3(kBlock), 0, w.stream, pol, sorted,
                           C, a, na, b, nb, w.bounds.as<const uint64_t>(), gkill, tmp, w.tile_cnt.as<uint32_t>());
    CG_HIP(hipGetLastError());
    hipLaunchKernelGGL(count_scan_kernel, dim3(nscan), dim3(kScanBlock), 0, w.stream,
                       w.tile_cnt.as<const uint32_t>(), ntiles, w.tile_off.as<uint64_t>(), d_count,
                       w.status.as<uint64_t>(), ticket, epoch, nscan, w.err());
    CG_HIP(hipGetLastError());
    // algorithmic traffic: candidates and both reference layers are read
    // once; the 8N bytes of the output are added by the caller once N is
    // known
    if (w.prof)
        w.prof->end(K_DEDUP, (double)sizeof(typename P::K) * (double)C + 8.0 * (double)(na + nb), (double)C);
    w.dedup_tiles = ntiles;
}

template <class P>
void dedup_gather_impl(P pol, const typename P::K *tmp, uint64_t *out, uint64_t out_cap, PipeWork &w,
                       typename P::K *rank_out = nullptr) {
    if (!w.dedup_tiles) return;
    if (w.prof) w.prof->begin(K_DEDUP);
    const uint32_t ntiles = (uint32_t)w.dedup_tiles;
    constexpr uint32_t tpb = (uint32_t)gather_tiles<P>();
    hipLaunchKernelGGL(gather_kernel<P>, dim3((ntiles + tpb - 1) / tpb), dim3(kBlock), 0,
                       w.stream, pol, tmp, w.tile_cnt.as<const uint32_t>(), w.tile_off.as<const uint64_t>(), ntiles,
                       out, out_cap, rank_out, w.err());
    CG_HIP(hipGetLastError());
    if (w.prof) w.prof->end(K_DEDUP, 0, 0);
}

}  // namespace

void launch_dedup_count(const uint64_t *sorted, uint64_t C, const uint64_t *a, uint64_t na,
                        const uint64_t *b, uint64_t nb, uint64_t *tmp, uint64_t *d_count,
                        PipeWork &w) {
    dedup_count_impl(PackedKeys{0}, sorted, C, a, na, b, nb, tmp, d_count, w);
}

void launch_dedup_gather(const uint64_t *tmp, uint64_t *out, uint64_t out_cap, PipeWork &w) {
    dedup_gather_impl(PackedKeys{0}, tmp, out, out_cap, w, (uint64_t *)nullptr);
}

void launch_dedup_count_ranked(int n, const uint32_t *sorted, uint64_t C, const uint64_t *a, uint64_t na,
                               const uint64_t *b, uint64_t nb, uint32_t *tmp, uint64_t *d_count,
                               PipeWork &w) {
    with_rank_n(n, [&](auto NN) {
        dedup_count_impl(RankedKeys<decltype(NN)::value>{n}, sorted, C, a, na, b, nb, tmp, d_count, w);
    });
}

void launch_dedup_gather_ranked(int n, const uint32_t *tmp, uint64_t *out, uint64_t out_cap, PipeWork &w,
                                uint32_t *rank_out) {
    with_rank_n(n, [&](auto NN) {
        dedup_gather_impl(RankedKeys<decltype(NN)::value>{n}, tmp, out, out_cap, w, rank_out);
    });
}

void launch_dedup_count_ranked_refs(int n, const uint32_t *sorted, uint64_t C, const uint32_t *a, uint64_t na,
                                    const uint32_t *b, uint64_t nb, uint32_t *tmp, uint64_t *d_count,
                                    PipeWork &w) {
    with_rank_n(n, [&](auto NN) {
        dedup_count_impl(RankedRefs<decltype(NN)::value>{n}, sorted, C, a, na, b, nb, tmp, d_count, w);
    });
}

void launch_dedup_count_ranked64(int n, const uint64_t *sorted, uint64_t C, const uint64_t *a, uint64_t na,
                                 const uint64_t *b, uint64_t nb, uint64_t *tmp, uint64_t *d_count, PipeWork &w) {
    with_rank64_n(n, [&](auto NN) {
        dedup_count_impl(Ranked64Keys<decltype(NN)::value>{n}, sorted, C, a, na, b, nb, tmp, d_count, w);
    });
}

void launch_dedup_gather_ranked64(int n, const uint64_t *tmp, uint64_t *out, uint64_t out_cap, PipeWork &w,
                                  uint64_t *rank_out) {
    with_rank64_n(n, [&](auto NN) {
        dedup_gather_impl(Ranked64Keys<decltype(NN)::value>{n}, tmp, out, out_cap, w, rank_out);
    });
}

void launch_dedup_count_ranked64_refs(int n, const uint64_t *sorted, uint64_t C, const uint64_t *a, uint64_t na,
                                      const uint64_t *b, uint64_t nb, uint64_t *tmp, uint64_t *d_count,
                                      PipeWork &w) {
    with_rank64_n(n, [&](auto NN) {
        dedup_count_impl(Ranked64Refs<decltype(NN)::value>{n}, sorted, C, a, na, b, nb, tmp, d_count, w);
    });
}

void launch_dedup(const uint64_t *sorted, uint64_t C, const uint64_t *a, uint64_t na,
                  const uint64_t *b, uint64_t nb, uint64_t *out, uint64_t out_cap,
                  uint64_t *tmp, uint64_t *d_count, PipeWork &w) {
    launch_dedup_count(sorted, C, a, na, b, nb, tmp, d_count, w);
    launch_dedup_gather(tmp, out, out_cap, w);
}

}  // namespace cg
