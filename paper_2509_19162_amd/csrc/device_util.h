// Device helpers for the gfx950 kernels: wave64 scans, decoupled look-back
// words, wave-cooperative searches in sorted global arrays.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cg {

constexpr int kWave = 64;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Number of set bits of `mask` below the calling lane (v_mbcnt pair).
__device__ __forceinline__ uint32_t mask_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t shfl_up64(uint64_t v, int d) {
    uint32_t lo = __shfl_up((uint32_t)v, d, kWave);
    uint32_t hi = __shfl_up((uint32_t)(v >> 32), d, kWave);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
    uint32_t lo = __shfl((uint32_t)v, src, kWave);
    uint32_t hi = __shfl((uint32_t)(v >> 32), src, kWave);
    return ((uint64_t)hi << 32) | lo;
}

// Inclusive prefix sum across the 64 lanes of a wave.
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint64_t t = shfl_up64(v, d);
        if (lane >= (uint32_t)d) v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan32(uint32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t t = __shfl_up(v, d, kWave);
        if (lane >= (uint32_t)d) v += t;
    }
    return v;
}

// Exclusive prefix sum over the threads of a block of WAVES waves.
// s_tmp must hold WAVES entries. Returns the calling thread's exclusive
// prefix; *total receives the block total. Contains __syncthreads().
template <int WAVES, class T>
__device__ __forceinline__ T block_excl_scan(T v, T *s_tmp, T *total) {
    const uint32_t lane = lane_id();
    const uint32_t wave = threadIdx.x / kWave;
    T incl;
    if constexpr (sizeof(T) == 8)
        incl = wave_incl_scan(v);
    else
        incl = wave_incl_scan32(v);
    if (lane == kWave - 1) s_tmp[wave] = incl;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        T x = s_tmp[w];
        if ((uint32_t)w < wave) off += x;
        tot += x;
    }
    *total = tot;
    __syncthreads();
    return off + incl - v;
}

// ---------------------------------------------------------------------------
// Decoupled look-back words: [63:48] epoch, [47:46] flag, [45:0] value.
// A word whose epoch differs from the launch's epoch reads as "not ready",
// so the array needs no clearing between launches.
// ---------------------------------------------------------------------------
constexpr uint32_t kFlagAggregate = 1;
constexpr uint32_t kFlagInclusive = 2;
constexpr uint64_t kValueMask = (1ull << 46) - 1;
constexpr uint32_t kSpinLimit = 1u << 24;
#ifndef CG_LB_DEPTH
#define CG_LB_DEPTH 1
#endif
constexpr int kLbDepth = CG_LB_DEPTH;  // predecessor words read in the first look-back round
#ifndef CG_LB_DEPTH_FAR
#define CG_LB_DEPTH_FAR 4
#endif
constexpr int kLbDepthFar = CG_LB_DEPTH_FAR;  // ... and in every later round

__device__ __forceinline__ uint64_t lb_word(uint32_t epoch, uint32_t flag, uint64_t v) {
    return ((uint64_t)epoch << 48) | ((uint64_t)flag << 46) | (v & kValueMask);
}

__device__ __forceinline__ void lb_store(uint64_t *p, uint64_t w) {
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t lb_load(const uint64_t *p) {
    return __hip_atomic_load(const_cast<uint64_t *>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

// One look-back round: reads the words of tiles t, t-1, ..., t-D+1 at once
// and adds the aggregates up to the first inclusive word, stopping at a
// word not yet published. Returns the tiles consumed; *done is set when an
// inclusive word was reached.
template <int D>
__device__ __forceinline__ int lb_round(const uint64_t *base, uint64_t stride, int64_t t, uint32_t epoch,
                                        uint64_t &excl, bool &done) {
    const uint64_t zero_incl = lb_word(epoch, kFlagInclusive, 0);
    uint64_t w[D];
#pragma unroll
    for (int u = 0; u < D; ++u) w[u] = (t - u >= 0) ? lb_load(base + (uint64_t)(t - u) * stride) : zero_incl;
    int used = 0;
#pragma unroll
    for (int u = 0; u < D; ++u) {
        if (done || used != u) break;
        if ((uint32_t)(w[u] >> 48) != epoch) break;
        excl += w[u] & kValueMask;
        ++used;
        if (((w[u] >> 46) & 3u) == kFlagInclusive) done = true;
    }
    return used;
}

// Exclusive prefix of tile `tile` from the words of tiles tile-1, tile-2, ...
// located at base[t * stride]. The first round reads kLbDepth predecessors
// (enough when a nearby tile has already published its inclusive word);
// later rounds read kLbDepthFar, so a long chain of aggregates costs few
// round trips. Tiles publish in ticket order, so every tile waited on is
// already running; the wait is still bounded: on overrun the error flag is
// raised and the (then meaningless) partial sum returned.
template <int kFirst = kLbDepth, int kFar = kLbDepthFar>
__device__ __forceinline__ uint64_t lb_lookback(const uint64_t *base, uint64_t stride,
                                                uint32_t tile, uint32_t epoch,
                                                uint32_t *err) {
    uint64_t excl = 0;
    int64_t t = (int64_t)tile - 1;
    uint32_t spins = 0;
    bool first = true;
    while (t >= 0) {
        bool done = false;
        const int used = first ? lb_round<kFirst>(base, stride, t, epoch, excl, done)
                               : lb_round<kFar>(base, stride, t, epoch, excl, done);
        if (done) break;
        t -= used;
        if (used == 0) {
            if (++spins > kSpinLimit) {
                atomicOr(err, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        } else {
            first = false;
        }
    }
    return excl;
}

// Wave-parallel look-back for one value per tile (words at base[t]): the 64
// lanes read the words of tiles tile-1 .. tile-64 at once, take the nearest
// inclusive word and add the aggregates before it; if all 64 are
// aggregates, they move 64 tiles back. Every lane of the wave must call it;
// all lanes return the same exclusive prefix. Bounded wait as above.
__device__ __forceinline__ uint64_t lb_lookback_wave(const uint64_t *base, uint32_t tile,
                                                     uint32_t epoch, uint32_t *err) {
    const uint32_t lane = lane_id();
    uint64_t excl = 0;
    int64_t top = (int64_t)tile - 1;  // highest tile not yet summed
    uint32_t spins = 0;
    while (top >= 0) {
        const int64_t t = top - (int64_t)lane;
        uint64_t w = 0;
        bool ready = true, incl = true;
        if (t >= 0) {
            w = lb_load(base + t);
            ready = (uint32_t)(w >> 48) == epoch;
            incl = ready && (((w >> 46) & 3u) == kFlagInclusive);
        }  // lanes before tile 0 act as an inclusive zero
        const uint64_t m_incl = __ballot(incl);
        const uint64_t m_ready = __ballot(ready);
        const uint32_t first = m_incl ? (uint32_t)__ffsll((unsigned long long)m_incl) - 1u : 64u;
        const uint64_t need = first >= 63u ? ~0ull : ((2ull << first) - 1ull);
        if ((m_ready & need) == need) {
            uint64_t v = (lane <= first && t >= 0) ? (w & kValueMask) : 0;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) v += shfl64(v, (lane + d) & 63) * (lane + d < 64);
            excl += shfl64(v, 0);
            if (first < 64u) break;
            top -= 64;
            continue;
        }
        if (++spins > kSpinLimit) {
            if (lane == 0) atomicOr(err, 1u);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return excl;
}

// ---------------------------------------------------------------------------
// Wave-cooperative search in a sorted global array: the first index i in
// [0, n] with !(a[i] < key) (upper == false) or !(a[i] <= key) (upper ==
// true). Every lane of the wave must call it with the same arguments; each
// round probes 64 evenly spaced elements.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t wave_search(const uint64_t *a, uint64_t n, uint64_t key,
                                                bool upper) {
    const uint32_t lane = lane_id();
    uint64_t lo = 0, hi = n;  // answer in [lo, hi]
    while (hi - lo > kWave) {
        const uint64_t step = (hi - lo + kWave - 1) / kWave;
        const uint64_t p = lo + (uint64_t)lane * step;
        bool pred = false;
        if (p < hi) {
            const uint64_t v = a[p];
            pred = upper ? (v <= key) : (v < key);
        }
        const uint32_t c = (uint32_t)__popcll(__ballot(pred));
        if (c == 0) return lo;
        const uint64_t nlo = lo + (uint64_t)(c - 1) * step + 1;
        const uint64_t cand = lo + (uint64_t)c * step;
        const uint64_t nhi = (c < (uint32_t)kWave && cand < hi) ? cand : hi;
        lo = nlo;
        hi = nhi;
    }
    const uint64_t p = lo + lane;
    bool pred = false;
    if (p < hi) {
        const uint64_t v = a[p];
        pred = upper ? (v <= key) : (v < key);
    }
    return lo + (uint64_t)__popcll(__ballot(pred));
}

}  // namespace cg
