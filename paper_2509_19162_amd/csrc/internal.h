// Internal declarations shared by the HIP kernels and the host runtime of
// libcayleygrowth.so. Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/cayleygrowth.h"

namespace cg {

// ---------------------------------------------------------------------------
// Errors: host code throws cg::Error; the C ABI turns it into a status code.
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void hip_check(hipError_t e, const char *what, const char *file, int line);
#define CG_HIP(x) ::cg::hip_check((x), #x, __FILE__, __LINE__)

// ---------------------------------------------------------------------------
// State keys. A state s (n <= 16 entries, each 0..15) is the uint64
//   key(s) = sum_i s[i] << 4*(n-1-i)
// so numeric order is lexicographic order. For every state of one orbit the
// last entry s[n-1] (nibble 0) follows from the others (the multiset of
// entries is fixed), so sorting and comparing on bits [4, 4n) is exact.
// Batched jobs put the job index above bit 4*16 - the tag bits - see batch.
// ---------------------------------------------------------------------------
constexpr uint64_t kSentinel = ~0ull;  // never a key: nibbles 15 everywhere

uint64_t pack_host(int n, const uint8_t *s);
void unpack_host(int n, uint64_t key, uint8_t *s);

// Byte-permute selectors of one generator (see make_gensel in expand.hip).
struct GenSel {
    uint32_t sel[8];
};
GenSel make_gensel(int n, const uint8_t *g);

// ---------------------------------------------------------------------------
// Per-kernel HIP-event profiling (CG_PROFILE).
// ---------------------------------------------------------------------------
enum KernelKind {
    K_EXPAND = 0,     // stand-alone permute-expand
    K_HIST = 1,       // one-read digit histograms of every sort pass
    K_SCAN = 2,       // digit offsets
    K_SORT_FUSED = 3, // first sort pass, candidates regenerated from frontier
    K_SORT = 4,       // later sort passes
    K_DEDUP = 5,      // unique + set difference + compaction
    K_AUX = 6,        // small bookkeeping kernels
    K_NUM = 7
};
const char *kernel_kind_name(int k);

struct Profiler {
    bool on = false;
    hipStream_t stream = nullptr;
    struct Pending {
        int kind;
        hipEvent_t a, b;
        double bytes, items;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    double total_ms[K_NUM] = {0};
    double bytes[K_NUM] = {0};
    double items[K_NUM] = {0};
    uint64_t launches[K_NUM] = {0};

    hipEvent_t get_event();
    // Record the start event of a launch of `kind` (no-op when off).
    void begin(int kind);
    // Record the end event; alg_bytes/items are this launch's algorithmic
    // traffic and processed keys.
    void end(int kind, double alg_bytes, double items);
    // After a stream synchronisation: fold finished launches into totals.
    void collect();
    ~Profiler();
};

// ---------------------------------------------------------------------------
// Device scratch of the layer pipeline (owned by an Engine, grown on demand).
// ---------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    int dev = 0;
    bool in_arena = false;
    hipStream_t stream = nullptr;  // the stream the owner uses the buffer on
    // Grow to at least `need` bytes (contents are not kept). Returns true if
    // the buffer was reallocated. Memory comes from the device arena.
    bool ensure(size_t need, double slack = 1.0);
    // ensure(), after freeing a buffer more than 1.25 x need + 64 MiB large
    // (a shared buffer shrinks when the jobs that grew it have left)
    bool fit(size_t need, double slack = 1.0) {
        if (p && bytes > need + need / 4 + (64u << 20)) release();
        return ensure(need, slack);
    }
    void release();
    // Exchanges the memory of two buffers (with where it came from; the
    // streams stay with their owners).
    void swap(DevBuf &o) {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
        std::swap(dev, o.dev);
        std::swap(in_arena, o.in_arena);
    }
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    template <class T>
    T *as() const { return static_cast<T *>(p); }
};

// cg_memory_stats: bytes held by the library's device buffers now and at
// most since the last reset, and the arenas' reserved size.
void memory_stats(cg_memory_stats_t *out, bool reset_peak);
// Frees the device arena (hipFree) when no buffer uses it
// (cg_release_cached_memory).
void release_cached_device_memory();
// Makes [p, p + bytes) the current device's arena (p == nullptr: back to an
// arena the library reserves itself). Throws CG_E_BUSY while buffers live
// in the current arena.
void set_workspace(void *p, size_t bytes);
// Statistics of a growth vector (stats.cpp); throws Error(CG_E_INVAL).
void growth_stats(const uint64_t *sizes, int num_layers, cg_growth_stats_t *out);

struct PipeWork {
    DevBuf hist;     // uint64 [kMaxPasses][256]: digit counts of every pass
    DevBuf base;     // uint64 [kMaxPasses][256]: exclusive digit offsets
    DevBuf small;    // uint32 tickets[32], err flag, uint64 counters
    DevBuf status;   // uint64 look-back words: tiles x 256 (sort), tiles (dedup)
    DevBuf bounds;   // uint64 [tiles][4]: reference-layer slices of dedup tiles
    DevBuf tile_cnt; // uint32 [tiles]: survivors per dedup tile
    DevBuf tile_off; // uint64 [tiles]: output offset per dedup tile
    DevBuf kill;     // uint8 [C]: candidates found in a reference layer
    DevBuf tcnt;     // uint32 [tiles][256]: digit counts per sort tile (reduce-then-scan)
    DevBuf toff;     // uint64 [tiles][256]: first output position per (tile, digit)
    DevBuf bsum;     // uint64 [tile runs][256]: digit sums per run of 1024 tiles
    uint32_t epoch = 0;  // 16-bit epoch of the look-back words
    uint32_t dedup_tiles = 0;  // tiles of the last launch_dedup_count
    hipStream_t stream = nullptr;
    Profiler *prof = nullptr;

    uint32_t *tickets() const { return small.as<uint32_t>(); }          // 32
    uint32_t *err() const { return small.as<uint32_t>() + 32; }        // 1
    uint64_t *counter() const { return small.as<uint64_t>() + 32; }    // 8 x u64
    void init(hipStream_t s);
    // Make room for `words` look-back words (new memory is cleared).
    void ensure_status(uint64_t words);
    // Epoch of the next look-back launch; on wrap-around the words are
    // cleared so that no stale word can carry a live epoch.
    uint32_t next_epoch();
};

constexpr int kMaxPasses = 8;

// ---- util.hip ---------------------------------------------------------------
// Zero a[0..na) (uint32) and b[0..nb) (uint64) with one small kernel.
void launch_clear(uint32_t *a, uint32_t na, uint64_t *b, uint32_t nb, hipStream_t s);

// ---- expand.hip -------------------------------------------------------------
void launch_expand(const uint64_t *frontier, uint64_t F, const GenSel *d_gsel,
                   int k, uint64_t *out, PipeWork &w);
void launch_pack(int n, const uint8_t *d_rows, uint64_t count, uint64_t *d_keys,
                 hipStream_t s);
void launch_unpack(int n, const uint64_t *d_keys, uint64_t count,
                   uint8_t *d_rows, hipStream_t s);

// ---- bits.hip (binary states: one bit per entry, n <= 64) ------------------
// Entry i of a 0/1 vector is bit n-1-i of its key.
uint64_t pack_bits_host(int n, const uint8_t *s);
// Per generator, ceil(n/8) tables of 256 words: the candidate bits that the
// set bits of one key byte move to (k * ceil(n/8) * 256 words).
std::vector<uint64_t> make_bit_tables(int n, const uint8_t *gens, int k);
// out[g*F + f] = frontier[f] . g for the k generators whose tables are at
// d_tables.
void launch_expand_bits(const uint64_t *frontier, uint64_t F, const uint64_t *d_tables, int n, int k,
                        uint64_t *out, PipeWork &w);
void launch_unpack_bits(int n, const uint64_t *d_keys, uint64_t count, uint8_t *d_rows, hipStream_t s);
// Key-range chunks of binary candidates: counts per range (key >> pshift,
// kChunkBins ranges) into d_hist, and the candidates of ranges [blo, bhi)
// appended to out through *cursor (at most cap; an overrun sets error bit 8).
void launch_prefix_hist_bits(const uint64_t *frontier, uint64_t F, const uint64_t *d_tables, int n, int k,
                             int pshift, unsigned long long *d_hist, PipeWork &w);
void launch_expand_filter_bits(const uint64_t *frontier, uint64_t F, const uint64_t *d_tables, int n, int k,
                               int pshift, uint32_t blo, uint32_t bhi, uint64_t *out, uint64_t cap,
                               unsigned long long *cursor, PipeWork &w);

// ---- radix_sort.hip ----------------------------------------------------------
int sort_passes(int bit_lo, int bit_hi);
// Sorts keys[0..count) on bits [bit_lo, bit_hi); returns the buffer that
// holds the result (keys or tmp). balanced: digits of equal widths (within
// one bit) instead of 8-bit digits from bit_lo up (same number of passes).
uint64_t *radix_sort(uint64_t *keys, uint64_t *tmp, uint64_t count, int bit_lo,
                     int bit_hi, PipeWork &w, bool balanced = false);
// Expands frontier[0..F) into the 32-bit ranks of the k*F candidates
// (n <= 12) while counting the digits of every pass, then sorts them on
// bits [0, rank_bits). Returns buf0 or buf1 (each k*F words). d_gfix
// (device, or null for full ranks): k bytes, per generator the first
// position from which it fixes every position (the ranks then reuse the
// parent's Lehmer digits from there on), followed at the next 4-byte
// boundary by k*n uint32 source shifts 4(n-1-g[i]).
uint32_t *expand_rank_sort(int n, const uint64_t *frontier, uint64_t F, const GenSel *d_gsel, const uint8_t *d_gfix,
                           int k, uint32_t *buf0, uint32_t *buf1, int rank_bits, PipeWork &w);
// The same for n = 13..16 with 64-bit ranks (full ranks, no incremental
// digits): sorts on bits [0, rank_bits), rank_bits = ceil(log2 n!).
uint64_t *expand_rank_sort64(int n, const uint64_t *frontier, uint64_t F, const GenSel *d_gsel, int k,
                             uint64_t *buf0, uint64_t *buf1, int rank_bits, PipeWork &w);
// The same for 32-bit keys (candidates under their lexicographic rank).
uint32_t *radix_sort32(uint32_t *keys, uint32_t *tmp, uint64_t count, int bit_lo,
                       int bit_hi, PipeWork &w);
// Expands frontier[0..F) by the k generators and sorts the k*F candidates on
// bits [bit_lo, bit_hi); the first pass regenerates candidates from the
// frontier instead of reading them. Returns buf0 or buf1 (each k*F keys).
uint64_t *expand_sort(const uint64_t *frontier, uint64_t F, const GenSel *d_gsel,
                      int k, uint64_t *buf0, uint64_t *buf1, int bit_lo,
                      int bit_hi, PipeWork &w);
uint64_t sort_status_words(uint64_t count);
uint64_t expand_sort_status_words(uint64_t F, int k);

// ---- dedup.hip ----------------------------------------------------------------
// Unique + set difference against sorted a[0..na) and b[0..nb) + compaction
// into out (room for out_cap keys; survivors beyond it are not written and
// raise the error flag); the number of kept keys lands in *d_count. tmp is
// scratch of C keys (it may be the sort's other buffer).
void launch_dedup(const uint64_t *sorted, uint64_t C, const uint64_t *a,
                  uint64_t na, const uint64_t *b, uint64_t nb, uint64_t *out,
                  uint64_t out_cap, uint64_t *tmp, uint64_t *d_count, PipeWork &w);
// The same in two halves, so the caller can size `out` once N is known:
// the count half leaves N in *d_count (survivors parked in tmp); the gather
// half moves them to out.
void launch_dedup_count(const uint64_t *sorted, uint64_t C, const uint64_t *a,
                        uint64_t na, const uint64_t *b, uint64_t nb, uint64_t *tmp,
                        uint64_t *d_count, PipeWork &w);
void launch_dedup_gather(const uint64_t *tmp, uint64_t *out, uint64_t out_cap, PipeWork &w);
// The same with candidates as 32-bit lexicographic ranks (n <= 12): the
// reference layers are ranked as they are read and survivors are written
// back as packed keys.
void launch_dedup_count_ranked(int n, const uint32_t *sorted, uint64_t C, const uint64_t *a,
                               uint64_t na, const uint64_t *b, uint64_t nb, uint32_t *tmp,
                               uint64_t *d_count, PipeWork &w);
// rank_out (optional): the survivors' ranks, beside the packed layer.
void launch_dedup_gather_ranked(int n, const uint32_t *tmp, uint64_t *out, uint64_t out_cap, PipeWork &w,
                                uint32_t *rank_out = nullptr);
// The same count with the reference layers given by their ranks.
void launch_dedup_count_ranked_refs(int n, const uint32_t *sorted, uint64_t C, const uint32_t *a, uint64_t na,
                                    const uint32_t *b, uint64_t nb, uint32_t *tmp, uint64_t *d_count,
                                    PipeWork &w);
// Dedup with candidates as 64-bit lexicographic ranks (n = 13..16): the
// reference layers (packed keys) are ranked as they are read; survivors are
// written back as packed keys.
void launch_dedup_count_ranked64(int n, const uint64_t *sorted, uint64_t C, const uint64_t *a, uint64_t na,
                                 const uint64_t *b, uint64_t nb, uint64_t *tmp, uint64_t *d_count, PipeWork &w);
// rank_out (optional): the survivors' 64-bit ranks, beside the packed layer.
void launch_dedup_gather_ranked64(int n, const uint64_t *tmp, uint64_t *out, uint64_t out_cap, PipeWork &w,
                                  uint64_t *rank_out = nullptr);
// The same count with the reference layers given by their 64-bit ranks.
void launch_dedup_count_ranked64_refs(int n, const uint64_t *sorted, uint64_t C, const uint64_t *a, uint64_t na,
                                      const uint64_t *b, uint64_t nb, uint64_t *tmp, uint64_t *d_count,
                                      PipeWork &w);
// Permute-expand into 32-bit ranks: out[g*F + f] = rank(key(s_f . g)).
void launch_expand_ranked(int n, const uint64_t *frontier, uint64_t F, const GenSel *d_gsel,
                          int k, uint32_t *out, PipeWork &w);
// True once the device's arena exists (buffers then grow to exact sizes).
bool arena_active();
// Largest block a DevBuf could get now: the arena's largest free range, or
// the device's free memory (hipMemGetInfo) when no arena exists.
size_t device_bytes_available();

// ---- key-range chunks (chunk.hip) ----
constexpr uint32_t kChunkBins = 4096;  // ranges by the top 12 bits of the sort key
// d_hist[b] += candidates whose sort value v has ((v >> pshift) & 4095) == b.
// ranked: v = 32-bit rank (n <= 12); else v = packed key.
void launch_prefix_hist(int n, bool ranked, const uint64_t *frontier, uint64_t F, const GenSel *d_gsel, int k,
                        int pshift, unsigned long long *d_hist, PipeWork &w);
// Appends the sort values of the candidates with range index in [blo, bhi)
// to out (uint32 when ranked, else uint64) through *cursor (at most cap).
void launch_expand_filter(int n, bool ranked, const uint64_t *frontier, uint64_t F, const GenSel *d_gsel, int k,
                          int pshift, uint32_t blo, uint32_t bhi, void *out, uint64_t cap,
                          unsigned long long *cursor, PipeWork &w);
uint64_t dedup_status_words(uint64_t C);

}  // namespace cg
