// Stable LSD radix sort, for gfx950, of 64-bit state keys on a bit range and
// of 32-bit lexicographic ranks (candidates of n <= 12 states).
//
// The growth step needs the candidates of a layer in sorted order so that
// repeats become neighbours and the set difference against the two previous
// (sorted) layers becomes a merge. The paper says only that its BFS is
// efficient and not straightforward (section "Examples and Tutorials"); the
// sort-based design here is this library's own.
//
// Structure (one-sweep LSD):
//   1. hist    one read of the keys computes the 8-bit digit histograms of
//              every pass at once (LDS counters, one flush per block); for
//              ranks the expand kernel counts them while it writes them;
//   2. scan    exclusive prefix of each pass's 256 digit counts;
//   3. pass p  each tile (4096 64-bit or 15360 32-bit keys) ranks its keys
//              per digit within each wave64 (an LDS word per digit collects
//              the mask of lanes sharing it, v_mbcnt gives the rank below),
//              publishes its per-digit counts as decoupled look-back words,
//              reads the exclusive prefix of the tiles before it, reorders
//              the tile in LDS by digit and writes runs of equal digits to
//              consecutive addresses. 64-bit passes run persistent blocks
//              that take tiles by ticket.
// Each pass reads and writes every key once (8 or 16 bytes per key).
//
// The first pass of expand_sort() regenerates the candidates from the
// frontier (permute-expand fused into the pass), so the unsorted candidate
// array is never written; expand_rank_sort() writes the candidates' ranks
// once, with the histograms of every pass.
#include <cstdlib>
#include <type_traits>

#include "internal.h"
#include "device_util.h"
#include "expand_device.h"
#include "perm_rank.h"

namespace cg {

namespace {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
// Keys per thread: 30 for 32-bit keys (512 threads, 15360-key tiles), 16
// for 64-bit keys (768 threads, below). Measured per tile with the
// real-time clock, a 64-bit tile spends 6 us loading and ranking, 11 us
// waiting for its predecessors' look-back words and 5.5 us reordering and
// writing. The wait is not the chain's own latency: wider look-back
// windows, and independent chains over segments of the keys, left the
// pass time as it was (or slowed it); it fills the time of the tiles in
// flight while the writes of the digit runs set the pace. 30 keys, their
// packed ranks and the look-back fit 80 VGPRs, which with the split LDS
// reorder below keeps 3 tiles resident per CU (32 keys need 88 VGPRs: 2).
#ifndef CG_SORT_IPT32
#define CG_SORT_IPT32 30
#endif
#ifndef CG_SORT_BLOCK32
#define CG_SORT_BLOCK32 512
#endif
// The LDS reorder of a sort tile runs in `split` rounds over a buffer of
// tile/split keys: less LDS per tile, more tiles resident per CU.
#ifndef CG_SORT_SPLIT32
#define CG_SORT_SPLIT32 2
#endif
#ifndef CG_SORT_SPLIT64
#define CG_SORT_SPLIT64 2
#endif
// 64-bit keys: 768 threads x 16 keys (12288-key tiles). A pass writes each
// digit's run of a tile contiguously; uniformly spread digits (64-bit
// ranks) leave runs of tile/256 keys whose cache lines at both ends are
// written partially, so longer tiles write more efficiently: S_16 LRX sort
// passes 866 ms at 4096-key tiles, 704 at 8192, 688 at 12288 (10240: 690);
// at one block per CU (more VGPRs) 16384-, 20480- and 24576-key tiles took
// 724, 694 and 697 ms, 768 x 32 keys 673 against 675 for 768 x 16.
#ifndef CG_SORT_IPT64
#define CG_SORT_IPT64 16
#endif
#ifndef CG_SORT_BLOCK64
#define CG_SORT_BLOCK64 768
#endif
template <class K>
struct TileOf {
    static constexpr int ipt = sizeof(K) == 4 ? CG_SORT_IPT32 : CG_SORT_IPT64;
    static constexpr int block = sizeof(K) == 4 ? CG_SORT_BLOCK32 : CG_SORT_BLOCK64;  // threads of a sort tile
    static constexpr int waves = block / kWave;
    static constexpr int tile = block * ipt;
    static constexpr int wave_seg = kWave * ipt;  // keys owned by one wave
    static constexpr int split = sizeof(K) == 4 ? CG_SORT_SPLIT32 : CG_SORT_SPLIT64;
    static constexpr int buf = tile / split;  // keys in the LDS reorder buffer
};
constexpr int kTile = TileOf<uint64_t>::tile;  // frontier states per tile of the fused first pass
// the shorter of the two tiles sizes the look-back words of a pass
constexpr int kTileMin = TileOf<uint32_t>::tile < kTile ? TileOf<uint32_t>::tile : kTile;
#ifndef CG_EXPAND_CONTIG
#define CG_EXPAND_CONTIG 1  // ranked-expand threads take consecutive frontier states
#endif
#ifndef CG_SORT_ROWS
#define CG_SORT_ROWS 1
#endif
constexpr int kRows = CG_SORT_ROWS;  // rows ranked per LDS round trip
// Look-back passes with persistent blocks, per key width (32-bit tiles are
// register-bound: the tile loop would push them into spills)
// look-back depths (first round, later rounds) of the 64-bit passes, whose
// tiles are shorter; the 32-bit passes use the defaults of device_util.h
#ifndef CG_LB_DEPTH64
#define CG_LB_DEPTH64 1
#endif
#ifndef CG_LB_DEPTH_FAR64
#define CG_LB_DEPTH_FAR64 3
#endif
#ifndef CG_SORT_PERSIST32
#define CG_SORT_PERSIST32 0
#endif
#ifndef CG_SORT_PERSIST64
#define CG_SORT_PERSIST64 1
#endif
// Streaming (non-temporal) key loads and scatter stores, per key width:
// for 64-bit keys they cut S_16 LRX sort passes by 6%; for 32-bit ranks
// the streaming stores cost 13% and the loads 1%, so those stay plain.
#ifndef CG_SORT_NT_LOAD32
#define CG_SORT_NT_LOAD32 0
#endif
#ifndef CG_SORT_NT_STORE32
#define CG_SORT_NT_STORE32 0
#endif
#ifndef CG_SORT_NT_LOAD64
#define CG_SORT_NT_LOAD64 1
#endif
#ifndef CG_SORT_NT_STORE64
#define CG_SORT_NT_STORE64 1
#endif
// Look-back words only for the values the pass's digit can take
#ifndef CG_LB_USED_DIGITS
#define CG_LB_USED_DIGITS 1
#endif
#ifndef CG_SORT_HALF_MASK
#define CG_SORT_HALF_MASK 1  // peer masks set and cleared by 32-bit halves
#endif

static_assert(kBlock == kRadix, "one thread per digit in the look-back");

// ---- key sources --------------------------------------------------------------
// A source maps (tile, index in tile) to a key and knows each tile's length.

template <class K>
struct ArraySrcT {
    using Key = K;
    const K *keys;
    uint64_t count;
    struct Tile {
        const K *p;
        uint32_t n;
        __device__ __forceinline__ K get(uint32_t i) const {
            if constexpr (sizeof(K) == 4 ? CG_SORT_NT_LOAD32 : CG_SORT_NT_LOAD64)
                return __builtin_nontemporal_load(p + i);
            else
                return p[i];
        }
    };
    static constexpr uint64_t kLen = TileOf<K>::tile;
    __device__ __forceinline__ Tile tile(uint32_t t) const {
        const uint64_t start = (uint64_t)t * kLen;
        const uint64_t left = count - start;
        return Tile{keys + start, (uint32_t)(left < kLen ? left : kLen)};
    }
    __host__ __device__ uint32_t tiles() const { return (uint32_t)((count + kLen - 1) / kLen); }
    void materialize(K *, PipeWork &) const {}
};
using ArraySrc = ArraySrcT<uint64_t>;

// A tile is one frontier block (kTile states) under one generator. Tiles
// are numbered so that the k tiles of a block are 8 apart: workgroups are
// dispatched round-robin over the 8 XCDs, so the tiles sharing a frontier
// block tend to run on one XCD and re-read the block from its L2. (Any
// numbering is correct; the candidates' initial order does not matter.)
constexpr uint32_t kXcds = 8;

struct ExpandSrc {
    using Key = uint64_t;
    const uint64_t *frontier;
    uint64_t F;
    const GenSel *gsel;
    uint32_t k;
    struct Tile {
        const uint64_t *p;
        GenSel sel;
        uint32_t n;
        __device__ __forceinline__ uint64_t get(uint32_t i) const { return apply_gensel(p[i], sel); }
    };
    __device__ __forceinline__ Tile tile(uint32_t t) const {
        const uint32_t nblocks = (uint32_t)((F + kTile - 1) / kTile);
        const uint32_t group = kXcds * k;            // tiles of 8 frontier blocks
        const uint32_t q = t / group;
        const uint32_t r = t - q * group;
        const uint32_t full = nblocks / kXcds;
        const uint32_t width = q < full ? kXcds : nblocks - full * kXcds;
        const uint32_t x = r % width;
        const uint32_t g = r / width;
        const uint32_t b = q * kXcds + x;
        const uint64_t start = (uint64_t)b * kTile;
        const uint64_t left = F - start;
        return Tile{frontier + start, gsel[g],
                    (uint32_t)(left < (uint64_t)kTile ? left : (uint64_t)kTile)};
    }
    __host__ __device__ uint32_t tiles() const {
        return (uint32_t)(((F + kTile - 1) / kTile) * (uint64_t)k);
    }
    void materialize(uint64_t *out, PipeWork &w) const { launch_expand(frontier, F, gsel, (int)k, out, w); }
};

struct PassDesc {
    int shift[kMaxPasses];
    uint32_t mask[kMaxPasses];
    int passes;
};

// ---- 1. histograms of all passes -------------------------------------------------
template <class Src>
__global__ __launch_bounds__(kBlock) void hist_kernel(Src src, uint32_t ntiles, PassDesc pd,
                                                      unsigned long long *__restrict__ ghist) {
    __shared__ uint32_t s_h[kMaxPasses][kRadix];
    for (int i = threadIdx.x; i < kMaxPasses * kRadix; i += kBlock) (&s_h[0][0])[i] = 0;
    __syncthreads();
    // Keys of neighbouring frontier states share their high digits, so each
    // thread counts runs of equal digits and adds a run with one atomic:
    // this keeps lanes from piling onto one LDS counter.
    uint32_t cur[kMaxPasses], run[kMaxPasses];
#pragma unroll
    for (int p = 0; p < kMaxPasses; ++p) {
        cur[p] = 0;
        run[p] = 0;
    }
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const auto T = src.tile(t);
        for (uint32_t i = threadIdx.x; i < T.n; i += kBlock) {
            const uint64_t key = (uint64_t)T.get(i);
#pragma unroll
            for (int p = 0; p < kMaxPasses; ++p) {
                if (p < pd.passes) {
                    const uint32_t d = (uint32_t)(key >> pd.shift[p]) & pd.mask[p];
                    if (d != cur[p]) {
                        if (run[p]) atomicAdd(&s_h[p][cur[p]], run[p]);
                        cur[p] = d;
                        run[p] = 1;
                    } else {
                        ++run[p];
                    }
                }
            }
        }
    }
#pragma unroll
    for (int p = 0; p < kMaxPasses; ++p)
        if (p < pd.passes && run[p]) atomicAdd(&s_h[p][cur[p]], run[p]);
    __syncthreads();
    for (int p = 0; p < pd.passes; ++p) {
        const uint32_t c = s_h[p][threadIdx.x];
        if (c) atomicAdd(&ghist[p * kRadix + threadIdx.x], (unsigned long long)c);
    }
}

// ---- 1b. ranked expand with the histograms of every pass --------------------------
// Each block takes a contiguous run of frontier states; every state is read
// once and mapped through all k generators, and the candidates' 32-bit
// ranks go out generator-major (out[g*F + f], coalesced per generator).
// The digits of every pass are counted on the way (runs of equal digits
// per thread are added with one LDS atomic), so the sort needs no separate
// histogram read.
#ifndef CG_EXPAND_IPT
#define CG_EXPAND_IPT 4
#endif
constexpr int kExpandIpt = CG_EXPAND_IPT;  // frontier states per thread and round
#ifndef CG_EXPAND_IPT_INCR
#define CG_EXPAND_IPT_INCR 6
#endif
// the same with incremental ranks (each state also holds its suffix sums)
constexpr int kExpandIptIncr = CG_EXPAND_IPT_INCR;
// Frontier state j of the calling thread within a round of kBlock*kExpandIpt
// states: consecutive per thread (CG_EXPAND_CONTIG, the default) or strided
// across the block. Consecutive states of the sorted frontier share their
// leading entries, so their candidates under one generator share high rank
// digits: the runs the histograms merge before each LDS atomic get long
// (S_12 pancake: expand 24.9 -> 15.7 ms).
template <int IPT = kExpandIpt>
__device__ __forceinline__ uint32_t expand_slot(int j) {
#if CG_EXPAND_CONTIG
    return threadIdx.x * IPT + (uint32_t)j;
#else
    return (uint32_t)j * kBlock + threadIdx.x;
#endif
}
// Digits of the low passes change from one candidate to the next: they go
// to LDS counters one by one. Higher digits come in runs (a thread's
// consecutive frontier states map to nearby ranks): each thread counts the
// run of its current digit and adds it when the digit changes.
#ifndef CG_HIST_DIRECT_PASSES
#define CG_HIST_DIRECT_PASSES 1
#endif

// Balanced digits: the last `extra` of the P passes take the one bit more
// (S_16: 45 bits as 7,7,7,8,8,8: sort passes 634 -> 616 ms against
// 8,8,8,7,7,7; S_12 ranks and binary states measured the same either way).
#ifndef CG_RANK_WIDE_LAST
#define CG_RANK_WIDE_LAST 1
#endif
__host__ __device__ constexpr bool wide_pass(int p, int P, int extra) {
    return CG_RANK_WIDE_LAST ? p >= P - extra : p < extra;
}

// Bits of the ranks of S_N (the smallest b with 2^b >= N!) and the sort
// passes over them, fixed at compile time for the ranked expand.
template <int N>
struct RankPasses {
    static constexpr uint64_t fact() {
        uint64_t f = 1;
        for (int i = 2; i <= N; ++i) f *= (uint64_t)i;
        return f;
    }
    static constexpr int bits() {
        int b = 0;
        while ((1ull << b) < fact()) ++b;
        return b;
    }
    static constexpr int passes = (bits() + kRadixBits - 1) / kRadixBits;
    // Balanced digits: bits() % passes of the passes take one bit more
    // (wide_pass; S_16: 45 bits as 7,7,7,8,8,8 rather than 8,8,8,8,8,5). A
    // digit of fewer bits leaves longer runs per tile, and the passes cost
    // less in sum: S_16 LRX sort passes 676 -> 655 ms. make_passes(.., true)
    // lays out the same passes.
    static constexpr int width(int p) {
        return passes == 0 ? 0 : bits() / passes + (wide_pass(p, passes, bits() % passes) ? 1 : 0);  // S_1: no passes
    }
    static constexpr int shift(int p) { return p == 0 ? 0 : shift(p - 1) + width(p - 1); }
    static constexpr uint32_t mask(int p) { return (1u << width(p)) - 1u; }
};

// Incremental ranks. The rank is sum_i c_i (n-1-i)! over the Lehmer digits
// c_i (perm_rank.h). A generator that fixes every position from m on keeps
// the set of values in front of each such position, so c_i of the
// candidate equals c_i of its parent for i >= m: only the digits before m
// are computed per candidate, and the parent's suffix sum of the rest is
// computed once per frontier state and shared by all generators.
constexpr uint32_t fact_c(int m) { return m <= 1 ? 1u : (uint32_t)m * fact_c(m - 1); }

// v * (N-1)! for a value v < N; (N-1)! = f << s with f < 2^24 so that the
// product is a 24-bit multiply (11! = 155925 << 8)
template <int N>
__device__ __forceinline__ uint32_t times_top_fact(uint32_t v) {
    constexpr uint32_t f = fact_c(N - 1);
    constexpr int s = f < (1u << 24) ? 0 : 8;
    static_assert((f >> s) < (1u << 24) && ((f >> s) << s) == f, "top factorial splits");
    return mad24<uint32_t>(v, f >> s, 0u) << s;
}

// Entry i of the candidate t = s.g is the nibble of the parent s at bit
// sh[i] (sh is the generator's row of shifts, the same across the wave).
__device__ __forceinline__ uint32_t nibble_at(uint32_t lo, uint32_t hi, uint32_t sh) {
    // sh is uniform: one select of the half, one bit-field extract
    return __builtin_amdgcn_ubfe(sh < 32u ? lo : hi, sh & 31u, 4u);
}

// sum of c_i(t) (N-1-i)! over the positions i < min(M, N-1) of t = s.g,
// reading t's entries from s through the shifts sh
template <int N, int M>
__device__ __forceinline__ uint32_t rank_prefix_from(uint64_t s, const uint32_t *__restrict__ sh) {
    constexpr int kEnd = M < N - 1 ? M : N - 1;
    const uint32_t lo = (uint32_t)s, hi = (uint32_t)(s >> 32);
    uint32_t unused = (1u << N) - 1u;
    const uint32_t v0 = nibble_at(lo, hi, sh[0]);
    uint32_t acc = times_top_fact<N>(v0);
    unused ^= 1u << v0;
#pragma unroll
    for (int i = 1; i < kEnd; ++i) {
        const uint32_t v = nibble_at(lo, hi, sh[i]);
        const uint32_t c = (uint32_t)__builtin_popcount(low_bits(unused, v));
        acc = mad24<uint32_t>(c, fact_c(N - 1 - i), acc);
        unused ^= 1u << v;
    }
    return acc;
}

// suffix sums sum_{i=m}^{N-2} c_i(s) (N-1-i)! of key s for m = 2..N-2, to
// dst[m-2]
template <int N>
__device__ __forceinline__ void rank_suffixes(uint64_t s, uint32_t *dst) {
    if constexpr (N >= 4) {
        uint32_t c[N];
        uint32_t unused = (1u << N) - 1u;
        unused ^= 1u << ((uint32_t)(s >> (4 * (N - 1))) & 15u);
#pragma unroll
        for (int i = 1; i < N - 1; ++i) {
            const uint32_t v = (uint32_t)(s >> (4 * (N - 1 - i))) & 15u;
            c[i] = (uint32_t)__builtin_popcount(low_bits(unused, v));
            unused ^= 1u << v;
        }
        uint32_t acc = 0;
#pragma unroll
        for (int m = N - 2; m >= 2; --m) {
            acc = mad24<uint32_t>(c[m], fact_c(N - 1 - m), acc);
            dst[m - 2] = acc;
        }
    }
}

// fn(integral_constant<int, M>) for the smallest M in [2, N] with m <= M
template <int N, int M = 2, class Fn>
__device__ __forceinline__ void with_prefix_len(int m, Fn &&fn) {
    if constexpr (M >= N) {
        fn(std::integral_constant<int, N>{});
    } else {
        if (m <= M)
            fn(std::integral_constant<int, M>{});
        else
            with_prefix_len<N, M + 1>(m, fn);
    }
}

// Rank type of S_N: 32 bits up to n = 12, 64 bits beyond (16! < 2^45).
template <int N>
using RankT = typename std::conditional<(N <= kRankMaxN), uint32_t, uint64_t>::type;

// gfix (null: full ranks): per generator, the first position from which it
// fixes every position (0 for the identity). Incremental ranks are built for
// 32-bit ranks only (n <= 12).
template <int N, bool Incr>
__global__ __launch_bounds__(kBlock) void expand_rank_hist_kernel(
    const uint64_t *__restrict__ frontier, uint64_t F, const GenSel *__restrict__ gsel,
    const uint8_t *__restrict__ gfix, int k, RankT<N> *__restrict__ out, uint64_t per_block,
    unsigned long long *__restrict__ ghist) {
    using R = RankT<N>;
    static_assert(!Incr || N <= kRankMaxN, "incremental ranks are 32-bit");
    constexpr int kIpt = Incr ? kExpandIptIncr : kExpandIpt;
    constexpr int kP = RankPasses<N>::passes;
    // the source shifts follow the k fix positions at the next 4-byte boundary
    const uint32_t *__restrict__ gsh =
        Incr ? reinterpret_cast<const uint32_t *>(gfix + (((uint32_t)k + 3u) & ~3u)) : nullptr;
    static_assert(kP <= kMaxPasses, "rank passes");
    constexpr int kSufRows = N > 4 ? N - 3 : 1;  // suffix sums for m = 2..N-2
    __shared__ uint32_t s_h[kMaxPasses][kRadix];
    for (int i = threadIdx.x; i < kMaxPasses * kRadix; i += kBlock) (&s_h[0][0])[i] = 0;
    __syncthreads();
    const uint64_t lo = (uint64_t)blockIdx.x * per_block;
    const uint64_t hi = lo + per_block < F ? lo + per_block : F;
    uint32_t cur[kMaxPasses], run[kMaxPasses];
#pragma unroll
    for (int p = 0; p < kMaxPasses; ++p) {
        cur[p] = 0;
        run[p] = 0;
    }
    // Every round but possibly the block's last is full: its body needs no
    // per-state bounds checks.
    auto round = [&](uint64_t base, auto guard) {
        constexpr bool kGuard = decltype(guard)::value;
        // full ranks permute the split state; incremental ones read the
        // few entries they need straight from the parent's key
        Nibbles st[Incr ? 1 : kIpt];
        uint64_t sk[Incr ? kIpt : 1];
        // per state, in registers: every use below indexes it with constants
        uint32_t suf[kIpt][Incr ? kSufRows : 1];
#pragma unroll
        for (int j = 0; j < kIpt; ++j) {
            const uint64_t f = base + expand_slot<kIpt>(j);
            const uint64_t key = !kGuard || f < hi ? frontier[f] : 0ull;
            if constexpr (Incr) {
                sk[j] = key;
                rank_suffixes<N>(key, suf[j]);
            } else {
                st[j] = split_nibbles(key);
            }
        }
        for (int g = 0; g < k; ++g) {
            R *o = out + (uint64_t)g * F;
            auto body = [&](auto MM) {
                constexpr int M = decltype(MM)::value;
#pragma unroll
                for (int j = 0; j < kIpt; ++j) {
                    const uint64_t f = base + expand_slot<kIpt>(j);
                    if (kGuard && f >= hi) continue;
                    R r;
                    if constexpr (!Incr) {
                        r = perm_rank_t<N, R>(apply_gensel(st[j], gsel[g]));
                    } else if constexpr (M <= N - 2) {
                        r = rank_prefix_from<N, M>(sk[j], gsh + (uint32_t)g * N) + suf[j][M - 2];
                    } else {
                        r = rank_prefix_from<N, M>(sk[j], gsh + (uint32_t)g * N);
                    }
                    o[f] = r;
#pragma unroll
                    for (int p = 0; p < kP; ++p) {
                        const uint32_t d = (uint32_t)(r >> RankPasses<N>::shift(p)) & RankPasses<N>::mask(p);
                        if (p < CG_HIST_DIRECT_PASSES) {
                            atomicAdd(&s_h[p][d], 1u);
                        } else {
                            const bool chg = d != cur[p];
                            if (chg) atomicAdd(&s_h[p][cur[p]], run[p]);  // run 0 before the first digit
                            run[p] = chg ? 1u : run[p] + 1u;
                            cur[p] = d;
                        }
                    }
                }
            };
            if constexpr (Incr)
                with_prefix_len<N>((int)gfix[g], body);  // uniform: one branch chain per generator
            else
                body(std::integral_constant<int, N>{});
        }
    };
    const uint64_t kRound = (uint64_t)kBlock * kIpt;
    uint64_t base = lo;
    for (; base + kRound <= hi; base += kRound) round(base, std::false_type{});
    if (base < hi) round(base, std::true_type{});
#pragma unroll
    for (int p = 0; p < kP; ++p)
        if (p >= CG_HIST_DIRECT_PASSES && run[p]) atomicAdd(&s_h[p][cur[p]], run[p]);
    __syncthreads();
#pragma unroll
    for (int p = 0; p < kP; ++p) {
        const uint32_t c = s_h[p][threadIdx.x];
        if (c) atomicAdd(&ghist[p * kRadix + threadIdx.x], (unsigned long long)c);
    }
}

// ---- 2. digit offsets ---------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void digit_scan_kernel(const unsigned long long *__restrict__ ghist,
                                                            unsigned long long *__restrict__ gbase) {
    __shared__ unsigned long long s_tmp[kWaves];
    const int p = blockIdx.x;
    const unsigned long long v = ghist[p * kRadix + threadIdx.x];
    unsigned long long tot;
    const unsigned long long ex = block_excl_scan<kWaves>(v, s_tmp, &tot);
    gbase[p * kRadix + threadIdx.x] = ex;
}

__global__ void clear_kernel(unsigned long long *__restrict__ a, uint32_t na,
                             uint32_t *__restrict__ b, uint32_t nb) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < na) a[i] = 0;
    if (i < nb) b[i] = 0;
}

// ---- 3. one scatter pass -----------------------------------------------------------------
// 6 waves per SIMD: at most 80 VGPRs (the register budget above)
#ifndef CG_SORT_WPE
#define CG_SORT_WPE 6
#endif
#define CG_SORT_ATTR __attribute__((amdgpu_waves_per_eu(CG_SORT_WPE)))
// The digit (k >> shift) & dmask, dmask = 2^width - 1: one bit-field
// extract for 32-bit keys (their digits never cross bit 32).
template <class K>
__device__ __forceinline__ uint32_t digit_of(K k, int shift, uint32_t dmask, uint32_t width) {
    if constexpr (sizeof(K) == 4)
        return __builtin_amdgcn_ubfe((uint32_t)k, (uint32_t)shift, width);
    else
        return (uint32_t)(k >> shift) & dmask;
}

// Lookback = true: tiles take tickets and chain their digit offsets by
// decoupled look-back. Lookback = false: tile = block index and each
// tile's digit offsets come precomputed in tile_off (reduce-then-scan).
template <class Src, bool Lookback>
__global__ __launch_bounds__(TileOf<typename Src::Key>::block) CG_SORT_ATTR void onesweep_kernel(
    Src src, typename Src::Key *__restrict__ out, uint64_t total, int shift, uint32_t dmask,
    const unsigned long long *__restrict__ digit_base, uint64_t *__restrict__ status,
    uint32_t *__restrict__ ticket, uint32_t epoch, uint32_t *__restrict__ err,
    const uint64_t *__restrict__ tile_off) {
    using K = typename Src::Key;
    constexpr int kIpt = TileOf<K>::ipt;
    constexpr int kTileK = TileOf<K>::tile;
    constexpr int kWaveSeg = TileOf<K>::wave_seg;
    constexpr int kBlk = TileOf<K>::block;
    constexpr int kWv = TileOf<K>::waves;
    constexpr int kSplit = TileOf<K>::split;
    constexpr int kBuf = TileOf<K>::buf;
    static_assert(kBlk >= kRadix, "one thread per digit in the look-back");
    static_assert(kIpt % 2 == 0 && kBuf * kSplit == kTileK, "two halves per register, whole rounds");
    __shared__ __align__(16) K s_keys[kBuf];
    __shared__ uint32_t s_cnt[kWv][kRadix];
    // per digit: its output start minus its start in the tile-sorted order,
    // one LDS read per key in the scatter; 64-bit keys keep the two starts
    // apart (folded, that pass spills a register)
    constexpr bool kFold = sizeof(K) == 4;
    __shared__ uint64_t s_gdelta[kRadix];
    __shared__ uint32_t s_lstart[kFold ? 1 : kRadix];
    __shared__ uint32_t s_scan[kWv];
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_next;

    // the digit masks of the ranking live in s_keys until the scatter
    uint64_t(*s_match)[kWv][kRadix] = reinterpret_cast<uint64_t(*)[kWv][kRadix]>(s_keys);
    static_assert(kRows * kWv * kRadix * sizeof(uint64_t) <= kBuf * sizeof(K),
                  "match words fit in the reorder buffer");
    static_assert(kIpt % kRows == 0, "rows per group divide the rows per thread");

    constexpr bool kPersist = Lookback && (sizeof(K) == 4 ? CG_SORT_PERSIST32 : CG_SORT_PERSIST64);
    const uint32_t dwidth = (uint32_t)__builtin_popcount(dmask);
    if (Lookback && threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
    // With look-back the blocks are persistent: each takes tiles in ticket
    // order until the tickets run out (every block ends on a ticket past the
    // last tile), which saves a block launch per tile. A block draws its next
    // ticket once the offsets of its current tile are published, and loads
    // that tile's keys while it writes out the last reorder round of the
    // current one (S_16 LRX sort passes 695 -> 678 ms). Every wait ends:
    // tickets are drawn only by running blocks, and the smallest tile whose
    // offsets are unpublished is either some block's current tile, whose
    // look-back waits only on smaller tiles, or some block's next tile, whose
    // block is writing out a tile that waits on nothing.
    const uint32_t ntiles = src.tiles();
    uint32_t next_tile = 0;
    bool preloaded = false;
    K key[kIpt];
    for (;;) {
    uint32_t tid = threadIdx.x;
    // an opaque copy of the thread index: addresses derived from it are
    // computed per tile, not hoisted out of the tile loop into registers
    if constexpr (kPersist) __asm__ volatile("" : "+v"(tid));
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wave = tid / kWave;
    for (int i = tid; i < kWv * kRadix; i += kBlk) (&s_cnt[0][0])[i] = 0;
    for (int i = tid; i < kRows * kWv * kRadix; i += kBlk) (&s_match[0][0][0])[i] = 0;
    __syncthreads();
    const uint32_t tile = Lookback ? (preloaded ? next_tile : s_tile) : blockIdx.x;
    if (kPersist && tile >= ntiles) break;  // same for the whole block
    const auto T = src.tile(tile);
    const uint32_t nvalid = T.n;

    // A short (last) tile is padded with all-ones keys, which rank as the
    // largest digit after every real key (index order); their count is
    // taken off that digit's published count, so no step below needs a
    // bounds check, and only the final write stops at nvalid.
    // Wave w owns keys [w*S, (w+1)*S) of the tile (S = kWaveSeg); item j of
    // lane l is key w*S + j*64 + l, so (wave, item, lane) order is index order and
    // the per-wave running counts give a stable rank.
    if (!preloaded) {
#pragma unroll
        for (int j = 0; j < kIpt; ++j) {
            const uint32_t i = wave * kWaveSeg + j * kWave + lane;
            key[j] = i < nvalid ? T.get(i) : (K)kSentinel;
        }
    }
    // Peers (lanes of this wave holding the same digit) come from LDS masks:
    // every lane ORs its lane bit into its digit's word, reads the words
    // back and clears its own. Rows are ranked kRows at a time, each row with
    // its own set of masks, so one LDS round trip serves kRows rows: a lane
    // of row r reads the masks of all kRows rows at its digit, which gives
    // the holders of that digit in earlier rows of the group and, for the
    // digit's first holder, the group's count. LDS instructions of one wave
    // are processed in issue order, so every read sees all ORs of its group
    // and no clear overtakes a read.
    // Item j's rank within the wave's digit run (< 2^16) sits in half j & 1
    // of rank2[j / 2]; the digit is taken from the key again when needed.
    uint32_t rank2[kIpt / 2];
    static_assert(kTileK <= (1 << 16), "ranks and tile positions fit in 16 bits");
#pragma unroll
    for (int j0 = 0; j0 < kIpt; j0 += kRows) {
        uint32_t d[kRows];
#pragma unroll
        for (int r = 0; r < kRows; ++r) d[r] = digit_of(key[j0 + r], shift, dmask, dwidth);
#if CG_SORT_HALF_MASK
        // a lane sets (and later clears) only its half-wave's 32-bit word
#pragma unroll
        for (int r = 0; r < kRows; ++r)
            atomicOr(reinterpret_cast<uint32_t *>(&s_match[r][wave][d[r]]) + (lane >> 5), 1u << (lane & 31));
#else
#pragma unroll
        for (int r = 0; r < kRows; ++r) atomicOr(&s_match[r][wave][d[r]], 1ull << lane);
#endif
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        uint64_t m[kRows][kRows];
        uint32_t old[kRows];
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
#pragma unroll
            for (int q = 0; q < kRows; ++q) m[r][q] = s_match[q][wave][d[r]];
            old[r] = s_cnt[wave][d[r]];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
#if CG_SORT_HALF_MASK
#pragma unroll
        for (int r = 0; r < kRows; ++r) reinterpret_cast<uint32_t *>(&s_match[r][wave][d[r]])[lane >> 5] = 0u;
#else
#pragma unroll
        for (int r = 0; r < kRows; ++r) s_match[r][wave][d[r]] = 0ull;
#endif
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            uint32_t before = mask_rank(m[r][r]);
            uint32_t total = 0;
            bool first = before == 0;
#pragma unroll
            for (int q = 0; q < kRows; ++q) {
                const uint32_t c = (uint32_t)__popcll(m[r][q]);
                total += c;
                if (q < r) {
                    before += c;
                    first = first && c == 0;
                }
            }
            const int j = j0 + r;
            if (j & 1)
                rank2[j >> 1] |= (old[r] + before) << 16;
            else
                rank2[j >> 1] = old[r] + before;
            // materialise the rank here: left to itself the compiler keeps
            // count and lane rank of every row apart until the scatter
            __asm__ volatile("" : "+v"(rank2[j >> 1]));
            if (first) s_cnt[wave][d[r]] = old[r] + total;
        }
    }
    __syncthreads();

    // thread tid < 256 owns digit tid: wave prefix, tile count, look-back
    uint32_t run = 0;
    if (tid < (uint32_t)kRadix) {
        const uint32_t d = tid;
#pragma unroll
        for (int w = 0; w < kWv; ++w) {
            const uint32_t c = s_cnt[w][d];
            s_cnt[w][d] = run;
            run += c;
        }
        if constexpr (Lookback) {
            // the padding keys all hold the largest digit: not published
            const uint32_t pub = run - (d == dmask ? (uint32_t)kTileK - nvalid : 0u);
            uint64_t *my = status + (uint64_t)tile * kRadix + d;
            uint64_t excl = 0;
            if (CG_LB_USED_DIGITS && d > dmask) {
                // a value this pass's digit never takes (7-bit digits: the
                // upper half, two whole waves): no word to publish or read
            } else if (tile == 0) {
                lb_store(my, lb_word(epoch, kFlagInclusive, pub));
            } else {
                lb_store(my, lb_word(epoch, kFlagAggregate, pub));
                excl = sizeof(K) == 4 ? lb_lookback(status + d, kRadix, tile, epoch, err)
                                      : lb_lookback<CG_LB_DEPTH64, CG_LB_DEPTH_FAR64>(status + d, kRadix, tile,
                                                                                      epoch, err);
                lb_store(my, lb_word(epoch, kFlagInclusive, excl + pub));
            }
            // the next tile's ticket, drawn once this tile's offsets are
            // published (before any scatter store of this wave is in flight)
            if (kPersist && tid == 0) s_next = atomicAdd(ticket, 1u);
            s_gdelta[d] = (uint64_t)digit_base[d] + excl;
        } else {
            s_gdelta[d] = tile_off[(uint64_t)tile * kRadix + d];
        }
    }
    {
        uint32_t tot;
        const uint32_t lstart = block_excl_scan<kWv>(run, s_scan, &tot);  // every thread takes part
        if (tid < (uint32_t)kRadix) {
            if constexpr (kFold)
                s_gdelta[tid] -= lstart;  // may wrap below zero; the sum below does not
            else
                s_lstart[tid] = lstart;
            // each wave's slot for this digit in the tile-sorted order
#pragma unroll
            for (int w = 0; w < kWv; ++w) s_cnt[w][tid] += lstart;
        }
    }
    __syncthreads();

    // rank within the wave's run -> position in the tile-sorted order
#pragma unroll
    for (int j = 0; j < kIpt; j += 2) {
        // digits taken afresh (opaque copies of the keys): reusing the ones
        // of the ranking would keep 32 of them live across the look-back
        K k0 = key[j], k1 = key[j + 1];
        __asm__ volatile("" : "+v"(k0), "+v"(k1));
        const uint32_t d0 = digit_of(k0, shift, dmask, dwidth);
        const uint32_t d1 = digit_of(k1, shift, dmask, dwidth);
        const uint32_t p0 = s_cnt[wave][d0] + (rank2[j >> 1] & 0xFFFFu);
        const uint32_t p1 = s_cnt[wave][d1] + (rank2[j >> 1] >> 16);
        rank2[j >> 1] = p0 | (p1 << 16);
    }
    // Reorder through LDS in rounds of kBuf positions, so that each digit's
    // run goes out as one contiguous write. Positions at or past nvalid hold
    // padding keys.
#pragma unroll
    for (int h = 0; h < kSplit; ++h) {
        const uint32_t lo = (uint32_t)h * kBuf;
        if (!kPersist && lo >= nvalid) break;  // same for the whole block
        const bool any = lo < nvalid;         // same for the whole block
        const bool last = h == kSplit - 1;
        if (h) __syncthreads();   // the previous round's readers are done
        if (any) {
#pragma unroll
            for (int j = 0; j < kIpt; ++j) {
                const uint32_t p = ((j & 1) ? rank2[j >> 1] >> 16 : rank2[j >> 1] & 0xFFFFu) - lo;
                if (p < (uint32_t)kBuf) s_keys[p] = key[j];
            }
        }
        __syncthreads();
        if (kPersist && last) {
            next_tile = s_next;
            preloaded = true;
            if (next_tile < ntiles) {
                const auto T2 = src.tile(next_tile);
#pragma unroll
                for (int j = 0; j < kIpt; ++j) {
                    const uint32_t i = wave * kWaveSeg + j * kWave + lane;
                    key[j] = i < T2.n ? T2.get(i) : (K)kSentinel;
                }
            }
        }
        const uint32_t cnt = !any ? 0u : nvalid - lo < (uint32_t)kBuf ? nvalid - lo : (uint32_t)kBuf;
        for (uint32_t i = tid; i < cnt; i += kBlk) {
            const K k = s_keys[i];
            const uint32_t d = digit_of(k, shift, dmask, dwidth);
            const uint64_t gpos = kFold ? s_gdelta[d] + (lo + i) : s_gdelta[d] + (lo + i - s_lstart[d]);
            if (gpos < total) {
                if constexpr (sizeof(K) == 4 ? CG_SORT_NT_STORE32 : CG_SORT_NT_STORE64)
                    __builtin_nontemporal_store(k, out + gpos);
                else
                    out[gpos] = k;
            } else {
                atomicOr(err, 2u);  // inconsistent offsets: never write out of bounds
            }
        }
    }
    if constexpr (!kPersist) break;
    __syncthreads();  // the reorder buffer is free
    }
}

// ---- 3b. reduce-then-scan: per-tile digit counts and their offsets ------------
// Same tiles (and the same load pattern) as the scatter pass; only the real
// keys of a short tile are counted.
template <class Src>
__global__ __launch_bounds__(TileOf<typename Src::Key>::block) void tile_count_kernel(Src src, int shift,
                                                                                     uint32_t dmask,
                                                                                     uint32_t *__restrict__ tcnt) {
    using K = typename Src::Key;
    constexpr int kIpt = TileOf<K>::ipt;
    constexpr int kWaveSeg = TileOf<K>::wave_seg;
    constexpr int kBlk = TileOf<K>::block;
    __shared__ uint32_t s_h[kRadix];
    const uint32_t tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    for (uint32_t i = tid; i < (uint32_t)kRadix; i += kBlk) s_h[i] = 0;
    __syncthreads();
    const auto T = src.tile(blockIdx.x);
    uint32_t cur = 0, run = 0;
#pragma unroll
    for (int j = 0; j < kIpt; ++j) {
        const uint32_t i = wave * kWaveSeg + j * kWave + lane;
        if (i < T.n) {
            const uint32_t d = (uint32_t)(T.get(i) >> shift) & dmask;
            if (d != cur) {
                if (run) atomicAdd(&s_h[cur], run);
                cur = d;
                run = 1;
            } else {
                ++run;
            }
        }
    }
    if (run) atomicAdd(&s_h[cur], run);
    __syncthreads();
    if (tid < (uint32_t)kRadix) tcnt[(uint64_t)blockIdx.x * kRadix + tid] = s_h[tid];
}

// Sums of each digit's counts over runs of `tb` tiles (one block per run).
__global__ __launch_bounds__(kBlock) void tile_colsum_kernel(const uint32_t *__restrict__ tcnt, uint32_t ntiles,
                                                             uint32_t tb, uint64_t *__restrict__ bsum) {
    const uint32_t b = blockIdx.x, d = threadIdx.x;
    const uint32_t t_end = min((b + 1) * tb, ntiles);
    uint64_t acc = 0;
    for (uint32_t t = b * tb; t < t_end; ++t) acc += tcnt[(uint64_t)t * kRadix + d];
    bsum[(uint64_t)b * kRadix + d] = acc;
}

// Exclusive scan of the run sums per digit, starting at the digit's base.
__global__ __launch_bounds__(kBlock) void bsum_scan_kernel(uint64_t *__restrict__ bsum, uint32_t nb,
                                                           const unsigned long long *__restrict__ digit_base) {
    const uint32_t d = threadIdx.x;
    uint64_t acc = digit_base[d];
    for (uint32_t b = 0; b < nb; ++b) {
        const uint64_t v = bsum[(uint64_t)b * kRadix + d];
        bsum[(uint64_t)b * kRadix + d] = acc;
        acc += v;
    }
}

// First output position of every (tile, digit).
__global__ __launch_bounds__(kBlock) void tile_offset_kernel(const uint32_t *__restrict__ tcnt, uint32_t ntiles,
                                                             uint32_t tb, const uint64_t *__restrict__ bsum,
                                                             uint64_t *__restrict__ toff) {
    const uint32_t b = blockIdx.x, d = threadIdx.x;
    const uint32_t t_end = min((b + 1) * tb, ntiles);
    uint64_t acc = bsum[(uint64_t)b * kRadix + d];
    for (uint32_t t = b * tb; t < t_end; ++t) {
        toff[(uint64_t)t * kRadix + d] = acc;
        acc += tcnt[(uint64_t)t * kRadix + d];
    }
}

// Passes of at most 8 bits over [bit_lo, bit_hi): from bit_lo up in 8-bit
// digits (the last one shorter), or with `balanced` as many passes with
// widths that differ by at most one bit (RankPasses lays out the same).
PassDesc make_passes(int bit_lo, int bit_hi, bool balanced = false) {
    PassDesc pd{};
    pd.passes = 0;
    if (balanced) {
        const int b = bit_hi - bit_lo;
        const int P = (b + kRadixBits - 1) / kRadixBits;
        int s = bit_lo;
        for (int p = 0; p < P; ++p) {
            const int bits = b / P + (wide_pass(p, P, b % P) ? 1 : 0);
            pd.shift[p] = s;
            pd.mask[p] = (1u << bits) - 1u;
            s += bits;
        }
        pd.passes = P;
        return pd;
    }
    for (int s = bit_lo; s < bit_hi; s += kRadixBits) {
        const int bits = (bit_hi - s) < kRadixBits ? (bit_hi - s) : kRadixBits;
        pd.shift[pd.passes] = s;
        pd.mask[pd.passes] = (1u << bits) - 1u;
        ++pd.passes;
    }
    return pd;
}

#ifndef CG_HIST_GRID_CAP
#define CG_HIST_GRID_CAP 8192  // blocks of the one-read histogram (grid-stride over tiles)
#endif
uint32_t hist_grid(uint32_t ntiles) {
    const uint32_t cap = CG_HIST_GRID_CAP;
    return ntiles < cap ? (ntiles ? ntiles : 1) : cap;
}

constexpr uint64_t kSkipCheckMin = 1ull << 22;

// Reduce-then-scan for passes over at least CG_SORT_RTS_MIN keys (default 0
// = never: on MI355X the look-back pass measured faster, 71 against 113 ms
// of sort passes for S_12 pancake).
bool use_reduce_then_scan(uint64_t count) {
    const char *e = std::getenv("CG_SORT_RTS_MIN");
    const uint64_t min_keys = e ? std::strtoull(e, nullptr, 10) : 0ull;
    return min_keys && count >= min_keys;
}

template <class Src>
typename Src::Key *run_sort(const Src &first_src, uint64_t count, typename Src::Key *buf0,
                            typename Src::Key *buf1, int bit_lo, int bit_hi, PipeWork &w, bool fused_first,
                            double first_read_bytes, const typename Src::Key *array_in,
                            bool hist_ready = false, bool skip_check = true, bool balanced = false) {
    using K = typename Src::Key;
    constexpr double kb = (double)sizeof(K);
    const PassDesc pd = make_passes(bit_lo, bit_hi, balanced);
    if (pd.passes > kMaxPasses) throw Error(-1, "sort bit range needs more than 8 passes");
    unsigned long long *hist = w.hist.as<unsigned long long>();
    unsigned long long *base = w.base.as<unsigned long long>();

    const uint32_t t0 = first_src.tiles();
    if (!hist_ready) {
        if (w.prof) w.prof->begin(K_AUX);
        hipLaunchKernelGGL(clear_kernel, dim3(8), dim3(256), 0, w.stream, hist,
                           (uint32_t)(kMaxPasses * kRadix), w.tickets(), 32u);
        CG_HIP(hipGetLastError());
        if (w.prof) w.prof->end(K_AUX, 0, 0);
        if (w.prof) w.prof->begin(K_HIST);
        hipLaunchKernelGGL(hist_kernel<Src>, dim3(hist_grid(t0)), dim3(kBlock), 0, w.stream, first_src,
                           t0, pd, hist);
        CG_HIP(hipGetLastError());
        if (w.prof) w.prof->end(K_HIST, first_read_bytes, (double)count);
    }

    if (w.prof) w.prof->begin(K_SCAN);
    hipLaunchKernelGGL(digit_scan_kernel, dim3(pd.passes), dim3(kBlock), 0, w.stream, hist, base);
    CG_HIP(hipGetLastError());
    if (w.prof) w.prof->end(K_SCAN, 0, 0);

    // A pass whose digit is the same for every key is the identity: for
    // large sorts the histograms come back to the host and such passes are
    // skipped (for example the unused high nibbles of short states in a
    // batched group).
    int keep[kMaxPasses];
    int nkeep = 0;
    if (skip_check && count >= kSkipCheckMin) {
        unsigned long long h[kMaxPasses * kRadix];
        CG_HIP(hipMemcpyAsync(h, hist, sizeof(unsigned long long) * kRadix * pd.passes, hipMemcpyDeviceToHost,
                              w.stream));
        CG_HIP(hipStreamSynchronize(w.stream));
        for (int p = 0; p < pd.passes; ++p) {
            bool trivial = false;
            for (int d = 0; d < kRadix; ++d) trivial = trivial || h[p * kRadix + d] == count;
            if (!trivial) keep[nkeep++] = p;
        }
    } else {
        for (int p = 0; p < pd.passes; ++p) keep[nkeep++] = p;
    }
    if (nkeep == 0) {
        if (!fused_first) return const_cast<K *>(array_in);
        first_src.materialize(buf0, w);  // contiguous, generator-major
        return buf0;
    }

    K *cur_out = buf0;
    const K *cur_in = nullptr;
    // Either one scatter pass with decoupled look-back, or reduce-then-scan
    // (a counting pass over the tiles, a scan of the counts, then the
    // scatter with known offsets).
    const bool rts = use_reduce_then_scan(count);
    auto pass = [&](const auto &src, int p, int kind, double bytes) {
        using S = typename std::decay<decltype(src)>::type;
        const uint32_t nt = src.tiles();
        if (w.prof) w.prof->begin(kind);
        if (rts) {
            const uint32_t tb = 1024;
            const uint32_t nb = (nt + tb - 1) / tb;
            w.tcnt.ensure((size_t)nt * kRadix * sizeof(uint32_t), 1.25);
            w.toff.ensure((size_t)nt * kRadix * sizeof(uint64_t), 1.25);
            w.bsum.ensure((size_t)nb * kRadix * sizeof(uint64_t), 1.25);
            hipLaunchKernelGGL(tile_count_kernel<S>, dim3(nt), dim3(TileOf<typename S::Key>::block), 0, w.stream, src,
                               pd.shift[p],
                               pd.mask[p], w.tcnt.as<uint32_t>());
            hipLaunchKernelGGL(tile_colsum_kernel, dim3(nb), dim3(kBlock), 0, w.stream, w.tcnt.as<const uint32_t>(),
                               nt, tb, w.bsum.as<uint64_t>());
            hipLaunchKernelGGL(bsum_scan_kernel, dim3(1), dim3(kBlock), 0, w.stream, w.bsum.as<uint64_t>(), nb,
                               base + p * kRadix);
            hipLaunchKernelGGL(tile_offset_kernel, dim3(nb), dim3(kBlock), 0, w.stream, w.tcnt.as<const uint32_t>(),
                               nt, tb, w.bsum.as<const uint64_t>(), w.toff.as<uint64_t>());
            hipLaunchKernelGGL((onesweep_kernel<S, false>), dim3(nt), dim3(TileOf<typename S::Key>::block), 0,
                               w.stream, src, cur_out, count,
                               pd.shift[p], pd.mask[p], base + p * kRadix, w.status.as<uint64_t>(), w.tickets() + p,
                               0u, w.err(), w.toff.as<const uint64_t>());
        } else {
            const uint32_t epoch = w.next_epoch();
            uint32_t grid = nt;
            if (sizeof(typename S::Key) == 4 ? CG_SORT_PERSIST32 : CG_SORT_PERSIST64) {
            // persistent blocks: as many as can be resident at once
            static const uint32_t resident = [] {
                int per_cu = 0, dev = 0, cus = 0;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, onesweep_kernel<S, true>,
                                                                  TileOf<typename S::Key>::block, 0) != hipSuccess ||
                    hipGetDevice(&dev) != hipSuccess ||
                    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
                    return 0u;
                return (uint32_t)(per_cu > 0 ? per_cu : 1) * (uint32_t)(cus > 0 ? cus : 1);
            }();
            if (resident && resident < grid) grid = resident;
            }
            hipLaunchKernelGGL((onesweep_kernel<S, true>), dim3(grid), dim3(TileOf<typename S::Key>::block), 0,
                               w.stream, src, cur_out, count,
                               pd.shift[p], pd.mask[p], base + p * kRadix, w.status.as<uint64_t>(), w.tickets() + p,
                               epoch, w.err(), (const uint64_t *)nullptr);
        }
        CG_HIP(hipGetLastError());
        if (w.prof) w.prof->end(kind, bytes, (double)count);
    };
    for (int q = 0; q < nkeep; ++q) {
        const int p = keep[q];
        if (q == 0) {
            pass(first_src, p, fused_first ? K_SORT_FUSED : K_SORT, first_read_bytes + kb * (double)count);
        } else {
            const ArraySrcT<K> s{cur_in, count};
            pass(s, p, K_SORT, 2.0 * kb * (double)count);
        }
        cur_in = cur_out;
        cur_out = (cur_out == buf0) ? buf1 : buf0;
    }
    return const_cast<K *>(cur_in);
}

}  // namespace

int sort_passes(int bit_lo, int bit_hi) { return make_passes(bit_lo, bit_hi).passes; }

uint64_t sort_status_words(uint64_t count) { return ((count + kTileMin - 1) / kTileMin) * kRadix; }

uint64_t expand_sort_status_words(uint64_t F, int k) {
    const uint64_t a = ((F + kTile - 1) / kTile) * (uint64_t)k * kRadix;
    const uint64_t b = sort_status_words(F * (uint64_t)k);
    return a > b ? a : b;
}

uint64_t *radix_sort(uint64_t *keys, uint64_t *tmp, uint64_t count, int bit_lo, int bit_hi,
                     PipeWork &w, bool balanced) {
    if (count <= 1 || bit_lo >= bit_hi) return keys;
    w.ensure_status(sort_status_words(count));
    const ArraySrc src{keys, count};
    // pass 0 reads `keys` and writes `tmp`; then they alternate
    return run_sort(src, count, tmp, keys, bit_lo, bit_hi, w, false, 8.0 * (double)count, keys, false, true,
                    balanced);
}

uint32_t *radix_sort32(uint32_t *keys, uint32_t *tmp, uint64_t count, int bit_lo, int bit_hi,
                       PipeWork &w) {
    if (count <= 1 || bit_lo >= bit_hi) return keys;
    w.ensure_status(sort_status_words(count));
    const ArraySrcT<uint32_t> src{keys, count};
    return run_sort(src, count, tmp, keys, bit_lo, bit_hi, w, false, 4.0 * (double)count, keys);
}

uint32_t *expand_rank_sort(int n, const uint64_t *frontier, uint64_t F, const GenSel *d_gsel, const uint8_t *d_gfix,
                           int k, uint32_t *buf0, uint32_t *buf1, int rank_bits, PipeWork &w) {
    const uint64_t C = F * (uint64_t)k;
    if (C == 0) return buf0;
    w.ensure_status(sort_status_words(C));
    unsigned long long *hist = w.hist.as<unsigned long long>();
    if (w.prof) w.prof->begin(K_AUX);
    hipLaunchKernelGGL(clear_kernel, dim3(8), dim3(256), 0, w.stream, hist, (uint32_t)(kMaxPasses * kRadix),
                       w.tickets(), 32u);
    CG_HIP(hipGetLastError());
    if (w.prof) w.prof->end(K_AUX, 0, 0);
    // rounds of kBlock*ipt states; at most 4096 blocks
    const bool incr = d_gfix && n >= 6;
    const uint64_t round = (uint64_t)kBlock * (incr ? kExpandIptIncr : kExpandIpt);
    const uint64_t rounds = (F + round - 1) / round;
    const uint64_t blocks = rounds < 4096 ? rounds : 4096;
    const uint64_t per_block = ((rounds + blocks - 1) / blocks) * round;
    const uint32_t grid = (uint32_t)((F + per_block - 1) / per_block);
    if (w.prof) w.prof->begin(K_EXPAND);
    with_rank_n(n, [&](auto NN) {
        constexpr int N = decltype(NN)::value;
        // the kernel's histograms follow the bits of S_N's ranks
        if (rank_bits != RankPasses<N>::bits()) throw Error(-1, "rank bits differ from those of n!");
        if (incr)
            hipLaunchKernelGGL((expand_rank_hist_kernel<N, true>), dim3(grid), dim3(kBlock), 0, w.stream, frontier,
                               F, d_gsel, d_gfix, k, buf0, per_block, hist);
        else
            hipLaunchKernelGGL((expand_rank_hist_kernel<N, false>), dim3(grid), dim3(kBlock), 0, w.stream, frontier,
                               F, d_gsel, (const uint8_t *)nullptr, k, buf0, per_block, hist);
    });
    CG_HIP(hipGetLastError());
    if (w.prof) w.prof->end(K_EXPAND, 8.0 * (double)F + 4.0 * (double)C, (double)C);
    if (rank_bits <= 0) return buf0;
    const ArraySrcT<uint32_t> src{buf0, C};
    // Ranks of a large layer's candidates spread over [0, n!): no pass is
    // the identity, so the histograms are not read back (no host sync); a
    // pass that is one anyway runs as an ordinary pass.
    return run_sort(src, C, buf1, buf0, 0, rank_bits, w, false, 4.0 * (double)C, buf0, true, false, true);
}

uint64_t *expand_rank_sort64(int n, const uint64_t *frontier, uint64_t F, const GenSel *d_gsel, int k,
                             uint64_t *buf0, uint64_t *buf1, int rank_bits, PipeWork &w) {
    const uint64_t C = F * (uint64_t)k;
    if (C == 0) return buf0;
    w.ensure_status(sort_status_words(C));
    unsigned long long *hist = w.hist.as<unsigned long long>();
    if (w.prof) w.prof->begin(K_AUX);
    hipLaunchKernelGGL(clear_kernel, dim3(8), dim3(256), 0, w.stream, hist, (uint32_t)(kMaxPasses * kRadix),
                       w.tickets(), 32u);
    CG_HIP(hipGetLastError());
    if (w.prof) w.prof->end(K_AUX, 0, 0);
    const uint64_t round = (uint64_t)kBlock * kExpandIpt;
    const uint64_t rounds = (F + round - 1) / round;
    const uint64_t blocks = rounds < 4096 ? rounds : 4096;
    const uint64_t per_block = ((rounds + blocks - 1) / blocks) * round;
    const uint32_t grid = (uint32_t)((F + per_block - 1) / per_block);
    if (w.prof) w.prof->begin(K_EXPAND);
    with_rank64_n(n, [&](auto NN) {
        constexpr int N = decltype(NN)::value;
        if (rank_bits != RankPasses<N>::bits()) throw Error(-1, "rank bits differ from those of n!");
        hipLaunchKernelGGL((expand_rank_hist_kernel<N, false>), dim3(grid), dim3(kBlock), 0, w.stream, frontier, F,
                           d_gsel, (const uint8_t *)nullptr, k, buf0, per_block, hist);
    });
    CG_HIP(hipGetLastError());
    if (w.prof) w.prof->end(K_EXPAND, 8.0 * (double)F + 8.0 * (double)C, (double)C);
    const ArraySrcT<uint64_t> src{buf0, C};
    // as for 32-bit ranks: every pass runs, the histograms stay on the device
    return run_sort(src, C, buf1, buf0, 0, rank_bits, w, false, 8.0 * (double)C, buf0, true, false, true);
}

uint64_t *expand_sort(const uint64_t *frontier, uint64_t F, const GenSel *d_gsel, int k,
                      uint64_t *buf0, uint64_t *buf1, int bit_lo, int bit_hi, PipeWork &w) {
    const uint64_t C = F * (uint64_t)k;
    if (C == 0) return buf0;
    if (bit_lo >= bit_hi) {
        launch_expand(frontier, F, d_gsel, k, buf0, w);
        return buf0;
    }
    w.ensure_status(expand_sort_status_words(F, k));
    const ExpandSrc src{frontier, F, d_gsel, (uint32_t)k};
    return run_sort(src, C, buf0, buf1, bit_lo, bit_hi, w, true, 8.0 * (double)F, nullptr);
}

}  // namespace cg
