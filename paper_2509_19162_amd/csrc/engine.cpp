// Single-job growth: layer-by-layer breadth-first search from the start
// vector (paper, section "Reminder on Cayley graphs, diameters, growth",
// definition of Growth; the search itself is the breadth-first one named in
// section "Examples and Tutorials").
//
// Per layer d, all on one stream:
//   expand_sort   candidates s.g for every s in L_d and every generator g,
//                 regenerated inside the first radix pass and sorted;
//   dedup         keep the first key of each run that is in neither L_d nor
//                 L_{d-1}, compacted in order into L_{d+1};
//   read N        8 bytes back to the host (the only host-device sync).
// The loop stops at an empty layer (complete), after max_layers layers, or
// after recording the first layer larger than max_frontier (truncated).
#include "engine.h"
#include "batch.h"
#include "bitmap.h"

#include "perm_rank.h"

#include <algorithm>
#include <cstdlib>
#include <memory>
#include <chrono>
#include <cstdio>
#include <cstring>

namespace cg {

double now_seconds() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

JobSpec canonicalize(const cg_job_t &job, bool batch) {
    JobSpec s;
    if (job.n < 1 || job.n > 64) throw Error(CG_E_INVAL, "n must be in 1..64 (above 16 with a 0/1 start vector)");
    // one bit per entry: asked for, or needed (more than 16 entries)
    s.binary = job.n > 16 || (job.flags & CG_BINARY_STATE);
    if (s.binary && !(job.flags & CG_START_STATE))
        throw Error(CG_E_INVAL, "binary states (n > 16 or CG_BINARY_STATE) need CG_START_STATE and a 0/1 start vector");
    if (s.binary && (job.flags & (CG_BITMASK | CG_SMALL_JOB)))
        throw Error(CG_E_INVAL, "binary states run on the sort path only");
    if (s.binary && batch) throw Error(CG_E_UNSUPPORTED, "batches and the serving queue use 4-bit states (n <= 16)");
    if (!job.gens || job.n_gens < 1) throw Error(CG_E_INVAL, "need at least one generator row");
    if (job.max_layers < 1) throw Error(CG_E_INVAL, "max_layers must be >= 1");
    const int n = job.n;
    s.n = n;
    s.max_layers = job.max_layers;
    s.max_frontier = job.max_frontier;
    s.flags = job.flags;
    if (batch && (job.flags & CG_KEEP_ALL_LAYERS)) throw Error(CG_E_INVAL, "batched jobs cannot keep all layers");
    if (batch && job.layers_out) throw Error(CG_E_INVAL, "batched jobs cannot export layers");
    s.layers_out = job.layers_out;
    s.layers_out_cap = job.layers_out ? job.layers_out_cap : 0;

    std::vector<std::vector<uint8_t>> rows;
    for (int g = 0; g < job.n_gens; ++g) {
        const uint8_t *r = job.gens + (size_t)g * n;
        bool seen[64] = {false};
        bool ident = true;
        for (int i = 0; i < n; ++i) {
            if (r[i] >= n || seen[r[i]]) {
                char buf[96];
                std::snprintf(buf, sizeof buf, "generator row %d is not a permutation of 0..%d", g, n - 1);
                throw Error(CG_E_INVAL, buf);
            }
            seen[r[i]] = true;
            ident = ident && r[i] == i;
        }
        if (ident) continue;
        std::vector<uint8_t> v(r, r + n);
        if (std::find(rows.begin(), rows.end(), v) == rows.end()) rows.push_back(v);
    }
    s.k = (int)rows.size();
    for (auto &r : rows) s.gens.insert(s.gens.end(), r.begin(), r.end());

    // closed under inverses?
    s.inverse_closed = true;
    for (auto &r : rows) {
        std::vector<uint8_t> inv(n);
        for (int i = 0; i < n; ++i) inv[r[i]] = (uint8_t)i;
        if (std::find(rows.begin(), rows.end(), inv) == rows.end()) {
            s.inverse_closed = false;
            break;
        }
    }
    if (!s.inverse_closed && !(job.flags & CG_ALLOW_DIRECTED))
        throw Error(CG_E_UNSUPPORTED,
                    "generating set is not closed under inverses (pass CG_ALLOW_DIRECTED)");

    if (job.flags & CG_START_STATE) {
        if (!job.start) throw Error(CG_E_INVAL, "CG_START_STATE without a start vector");
        for (int i = 0; i < n; ++i) {
            if (job.start[i] > 15) throw Error(CG_E_INVAL, "start entries must be 0..15");
            if (s.binary && job.start[i] > 1) throw Error(CG_E_INVAL, "binary states need a 0/1 start vector");
            s.start[i] = job.start[i];
        }
    } else {
        for (int i = 0; i < n; ++i) s.start[i] = (uint8_t)i;
    }
    // orbit size bound: multinomial n! / prod(mult!) (at most C(64, 32) <
    // 2^61 for binary states, 16! for 4-bit ones)
    int mult[16] = {0};
    for (int i = 0; i < n; ++i) mult[s.start[i]]++;
    unsigned __int128 b = 1;
    int placed = 0;
    for (int v = 0; v < 16; ++v) {
        for (int j = 1; j <= mult[v]; ++j) {
            ++placed;
            b = b * (unsigned)placed / (unsigned)j;  // exact: running binomial products
        }
    }
    s.orbit_bound = (uint64_t)b;
    return s;
}

Engine::Engine(hipStream_t user_stream) {
    if (user_stream) {
        stream_ = user_stream;
    } else {
        CG_HIP(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking));
        own_stream_ = true;
    }
    w_.init(stream_);
    for (DevBuf *b : {&gsel_, &cand0_, &cand1_, &lay_[0], &lay_[1], &lay_[2], &arena_, &stage_, &chunk_hist_, &vis_[0],
                      &vis_[1], &rk_[0], &rk_[1], &rk_[2]})
        b->stream = stream_;
    prof_.stream = stream_;
    CG_HIP(hipHostMalloc((void **)&host_small_, kHostSmallBytes, hipHostMallocDefault));
}

Engine::~Engine() {
    delete wg_;
    if (host_small_) (void)hipHostFree(host_small_);
    // buffers go back to the device cache while their stream still exists
    for (DevBuf *b : {&gsel_, &cand0_, &cand1_, &lay_[0], &lay_[1], &lay_[2], &arena_, &stage_, &chunk_hist_,
                      &vis_[0], &vis_[1], &rk_[0], &rk_[1], &rk_[2]})
        b->release();
    for (DevBuf *b : {&w_.hist, &w_.base, &w_.small, &w_.status, &w_.bounds, &w_.tile_cnt, &w_.tile_off,
                      &w_.kill, &w_.tcnt, &w_.toff, &w_.bsum})
        b->release();
    if (own_stream_) {
        (void)hipStreamSynchronize(stream_);
        (void)hipStreamDestroy(stream_);
    }
}

uint64_t Engine::device_bytes() const {
    uint64_t b = 0;
    for (const DevBuf *x : {&gsel_, &cand0_, &cand1_, &lay_[0], &lay_[1], &lay_[2], &arena_, &stage_, &chunk_hist_,
                            &vis_[0], &vis_[1], &rk_[0], &rk_[1], &rk_[2]})
        b += x->bytes;
    for (const DevBuf *x : {&w_.hist, &w_.base, &w_.small, &w_.status, &w_.bounds, &w_.tile_cnt, &w_.tile_off,
                            &w_.kill, &w_.tcnt, &w_.toff, &w_.bsum})
        b += x->bytes;
    if (wg_) b += wg_->device_bytes();
    return b;
}

void Engine::release_buffers() {
    if (wg_) wg_->release();
    for (DevBuf *x : {&gsel_, &cand0_, &cand1_, &lay_[0], &lay_[1], &lay_[2], &arena_, &stage_, &chunk_hist_,
                      &vis_[0], &vis_[1], &rk_[0], &rk_[1], &rk_[2]})
        x->release();
    // the pipeline's small buffers stay (init sized them); the large ones go
    for (DevBuf *x : {&w_.status, &w_.bounds, &w_.tile_cnt, &w_.tile_off, &w_.kill, &w_.tcnt, &w_.toff, &w_.bsum})
        x->release();
    w_.epoch = 0;
}

uint64_t Engine::read_counter() {
    // the error flag and the counter lie in one small device buffer: one
    // copy brings both
    const char *lo = (const char *)w_.err();
    const size_t span = (size_t)((const char *)(w_.counter() + 1) - lo);
    static_assert(kHostSmallBytes >= 256, "the flag-to-counter span fits");
    if ((const char *)w_.counter() < lo || span > kHostSmallBytes) throw Error(-1, "counter layout");
    CG_HIP(hipMemcpyAsync(host_small_, lo, span, hipMemcpyDeviceToHost, stream_));
    CG_HIP(hipStreamSynchronize(stream_));
    const char *h = (const char *)host_small_;
    uint32_t err;
    uint64_t count;
    std::memcpy(&err, h, sizeof err);
    std::memcpy(&count, h + ((const char *)w_.counter() - lo), sizeof count);
    if (err != 0) throw Error(CG_E_DEVICE, "kernel error flag set (look-back bound or offset check)");
    return count;
}

void Engine::export_layer(const JobSpec &spec, const uint64_t *d_keys, uint64_t count,
                          uint64_t &written) {
    if (!spec.layers_out || written >= spec.layers_out_cap) {
        written += count;
        return;
    }
    const uint64_t take = std::min(count, spec.layers_out_cap - written);
    stage_.ensure(take * (uint64_t)spec.n + 64, 1.25);
    if (spec.binary)
        launch_unpack_bits(spec.n, d_keys, take, stage_.as<uint8_t>(), stream_);
    else
        launch_unpack(spec.n, d_keys, take, stage_.as<uint8_t>(), stream_);
    CG_HIP(hipMemcpyAsync(spec.layers_out + written * spec.n, stage_.p, take * spec.n,
                          hipMemcpyDeviceToHost, stream_));
    CG_HIP(hipStreamSynchronize(stream_));
    written += count;
}

void fill_kstats(const Profiler &p, cg_result_t *res) {
    res->n_kstats = 0;
    if (!p.on) return;
    for (int k = 0; k < K_NUM && res->n_kstats < CG_KSTAT_MAX; ++k) {
        if (!p.launches[k]) continue;
        cg_kstat_t &s = res->kstats[res->n_kstats++];
        std::memset(&s, 0, sizeof s);
        std::snprintf(s.name, sizeof s.name, "%s", kernel_kind_name(k));
        s.launches = p.launches[k];
        s.total_ms = p.total_ms[k];
        s.alg_bytes = p.bytes[k];
        s.items = p.items[k];
    }
}

// CG_CHUNK_CANDIDATES (tests) forces chunks of at most that many candidates.
uint64_t Engine::forced_chunk(uint64_t C) {
    if (const char *e = std::getenv("CG_CHUNK_CANDIDATES")) {
        const uint64_t v = std::strtoull(e, nullptr, 10);
        if (v > 0) return std::min<uint64_t>(v, C);
    }
    return C;
}

// Candidates per chunk when a layer's candidate arrays do not fit: two
// arrays of that many keys in 60% of the largest free block, the rest left
// for the chunks' survivors.
uint64_t Engine::chunk_capacity(uint64_t C, size_t key_bytes) {
    const double avail = (double)device_bytes_available();
    const uint64_t fit = (uint64_t)(avail * 0.6 / (double)(2 * key_bytes));
    return std::max<uint64_t>(1, std::min<uint64_t>(fit, C));
}

// One layer in key-range chunks (see chunk.hip). Survivors of each chunk
// are compacted into a buffer of their own, then concatenated in key order
// into dst (keep-all: the arena slot of the new layer, capacity out_cap) or
// into lay_[in] at its exact size. Returns the new layer's size.
uint64_t Engine::run_chunked(bool ranked, int n, const uint64_t *Ld, uint64_t F, const uint64_t *Ra, uint64_t na,
                             const uint64_t *Rb, uint64_t nb, int k, uint64_t cap, int rank_bits, int bit_lo,
                             int bit_hi, uint64_t *dst, uint64_t out_cap, uint64_t room, int in) {
    const int pshift = ranked ? std::max(0, rank_bits - 12) : std::max(bit_lo, bit_hi - 12);
    const size_t kb = ranked ? sizeof(uint32_t) : sizeof(uint64_t);
    chunk_hist_.stream = stream_;
    chunk_hist_.ensure(kChunkBins * sizeof(uint64_t));
    launch_clear(nullptr, 0, chunk_hist_.as<uint64_t>(), kChunkBins, stream_);
    if (binary_)
        launch_prefix_hist_bits(Ld, F, gsel_.as<uint64_t>(), n, k, pshift, chunk_hist_.as<unsigned long long>(), w_);
    else
        launch_prefix_hist(n, ranked, Ld, F, gsel_.as<GenSel>(), k, pshift, chunk_hist_.as<unsigned long long>(),
                           w_);
    std::vector<uint64_t> h(kChunkBins);
    CG_HIP(hipMemcpyAsync(h.data(), chunk_hist_.p, sizeof(uint64_t) * kChunkBins, hipMemcpyDeviceToHost, stream_));
    CG_HIP(hipStreamSynchronize(stream_));
    // consecutive ranges grouped while they fit
    struct Chunk {
        uint32_t lo, hi;
        uint64_t count;
    };
    std::vector<Chunk> chunks;
    uint64_t cap_used = 0;
    for (uint32_t b = 0; b < kChunkBins; ++b) {
        if (h[b] > cap) throw Error(CG_E_NOMEM, "one key range holds more candidates than fit in device memory");
        if (chunks.empty() || chunks.back().count + h[b] > cap) chunks.push_back({b, b, 0});
        chunks.back().hi = b + 1;
        chunks.back().count += h[b];
        cap_used = std::max(cap_used, chunks.back().count);
    }
    cand0_.ensure(std::max<uint64_t>(cap_used, 1) * kb);
    cand1_.ensure(std::max<uint64_t>(cap_used, 1) * kb);
    std::vector<std::unique_ptr<DevBuf>> parts;
    std::vector<uint64_t> part_n;
    uint64_t total = 0;
    unsigned long long *cursor = (unsigned long long *)(w_.counter() + 1);
    for (const Chunk &c : chunks) {
        if (!c.count) continue;
        launch_clear(nullptr, 0, w_.counter() + 1, 1, stream_);
        if (binary_)
            launch_expand_filter_bits(Ld, F, gsel_.as<uint64_t>(), n, k, pshift, c.lo, c.hi, cand0_.as<uint64_t>(),
                                      c.count, cursor, w_);
        else
            launch_expand_filter(n, ranked, Ld, F, gsel_.as<GenSel>(), k, pshift, c.lo, c.hi, cand0_.p, c.count,
                                 cursor, w_);
        uint64_t nj = 0;
        auto part = std::make_unique<DevBuf>();
        part->stream = stream_;
        if (ranked) {
            uint32_t *c0 = cand0_.as<uint32_t>(), *c1 = cand1_.as<uint32_t>();
            uint32_t *sorted = radix_sort32(c0, c1, c.count, 0, rank_bits, w_);
            uint32_t *scratch = sorted == c0 ? c1 : c0;
            launch_dedup_count_ranked(n, sorted, c.count, Ra, na, Rb, nb, scratch, w_.counter(), w_);
            nj = read_counter();
            if (nj > c.count) throw Error(CG_E_DEVICE, "chunk size out of range (device error)");
            if (nj) {
                part->ensure(nj * sizeof(uint64_t));
                launch_dedup_gather_ranked(n, scratch, part->as<uint64_t>(), nj, w_);
            }
        } else {
            uint64_t *c0 = cand0_.as<uint64_t>(), *c1 = cand1_.as<uint64_t>();
            uint64_t *sorted = radix_sort(c0, c1, c.count, bit_lo, bit_hi, w_, binary_);
            uint64_t *scratch = sorted == c0 ? c1 : c0;
            launch_dedup_count(sorted, c.count, Ra, na, Rb, nb, scratch, w_.counter(), w_);
            nj = read_counter();
            if (nj > c.count) throw Error(CG_E_DEVICE, "chunk size out of range (device error)");
            if (nj) {
                part->ensure(nj * sizeof(uint64_t));
                launch_dedup_gather(scratch, part->as<uint64_t>(), nj, w_);
            }
        }
        if (nj) {
            parts.push_back(std::move(part));
            part_n.push_back(nj);
            total += nj;
        }
    }
    if (total > room) throw Error(CG_E_DEVICE, "layer size out of range (device error)");
    // the candidate arrays (the largest buffers) are done with: the new
    // layer and the chunks' survivors must fit beside the window
    cand0_.release();
    cand1_.release();
    if (!dst) {
        lay_[in].ensure(std::max<uint64_t>(total, 1) * sizeof(uint64_t), 1.25);
        dst = lay_[in].as<uint64_t>();
    } else if (total > out_cap) {
        throw Error(CG_E_DEVICE, "layer larger than its slot (device error)");
    }
    uint64_t off = 0;
    for (size_t i = 0; i < parts.size(); ++i) {
        CG_HIP(hipMemcpyAsync(dst + off, parts[i]->p, part_n[i] * sizeof(uint64_t), hipMemcpyDeviceToDevice,
                              stream_));
        off += part_n[i];
    }
    CG_HIP(hipStreamSynchronize(stream_));
    for (auto &p : parts) p->release();
    return total;
}

void Engine::run(const JobSpec &spec, cg_result_t *res) {
    const double t0 = now_seconds();
    uint64_t *sizes = res->layer_sizes;
    std::memset(sizes, 0, sizeof(uint64_t) * (size_t)spec.max_layers);
    res->status = CG_OK;
    res->num_layers = 1;
    res->states_expanded = 0;
    res->candidates = 0;
    res->device_ms = 0;
    res->n_kstats = 0;
    sizes[0] = 1;

    prof_.on = (spec.flags & CG_PROFILE) != 0;
    for (int i = 0; i < K_NUM; ++i) {
        prof_.total_ms[i] = prof_.bytes[i] = prof_.items[i] = 0;
        prof_.launches[i] = 0;
    }
    w_.prof = prof_.on ? &prof_ : nullptr;

    if (spec.flags & CG_BITMASK) {
        run_bitmask(spec, res, stream_);
        return;
    }
    if (spec.flags & CG_SMALL_JOB) {
        if (!wg_eligible(spec))
            throw Error(CG_E_INVAL, "CG_SMALL_JOB needs n <= 10, a permutation start, at most 128 generators "
                                    "and no layer export");
        if (!wg_) wg_ = new WgRunner(stream_);
        std::vector<WgItem> one{{&spec, res}};
        WgTuning t;
        t.block = spec.n >= 10 ? 1024 : (spec.n == 9 ? 512 : 256);
        wg_->run(one, t, t0);
        return;
    }
    const int n = spec.n, k = spec.k;
    const bool keep_all = (spec.flags & CG_KEEP_ALL_LAYERS) != 0;
    // A set not closed under inverses can reach any earlier layer, so the
    // new layer is taken against every state seen so far: a sorted visited
    // array into which each new layer is merged.
    const bool directed = !spec.inverse_closed;

    hipEvent_t ev0, ev1;
    CG_HIP(hipEventCreate(&ev0));
    CG_HIP(hipEventCreate(&ev1));
    CG_HIP(hipEventRecord(ev0, stream_));

    uint64_t written = 0;
    const bool binary = spec.binary;
    binary_ = binary;
    const uint64_t key0 = binary ? pack_bits_host(n, spec.start) : pack_host(n, spec.start);
    if (binary) {
        // per generator, the byte tables of its bit permutation
        const std::vector<uint64_t> t = make_bit_tables(n, spec.gens.data(), k);
        gsel_.ensure(std::max<size_t>(t.size(), 1) * sizeof(uint64_t));
        if (!t.empty())
            CG_HIP(hipMemcpyAsync(gsel_.p, t.data(), t.size() * sizeof(uint64_t), hipMemcpyHostToDevice, stream_));
    }

    // generator selectors, followed by each generator's first position
    // from which it fixes every position
    std::vector<GenSel> hsel(k > 0 && !binary ? k : 1);
    std::vector<uint8_t> hfix(hsel.size(), 0);
    int moved = 0;  // Lehmer digits an incremental rank computes per state and all generators
    for (int g = 0; g < k && !binary; ++g) {
        const uint8_t *row = spec.gens.data() + (size_t)g * n;
        hsel[g] = make_gensel(n, row);
        for (int p = 0; p < n; ++p)
            if (row[p] != p) hfix[g] = (uint8_t)(p + 1);
        moved += std::min(std::max<int>(hfix[g], 2), n - 1) - 1;
    }
    // then, at the next 4-byte boundary, each generator's n source shifts:
    // entry i of candidate s.g is the nibble of s at bit 4(n-1-g[i])
    std::vector<uint32_t> hsh(binary ? 0 : hsel.size() * (size_t)n, 0);
    for (int g = 0; g < k && !binary; ++g)
        for (int i = 0; i < n; ++i) hsh[(size_t)g * n + i] = 4u * (uint32_t)(n - 1 - spec.gens[(size_t)g * n + i]);
    const size_t sel_bytes = sizeof(GenSel) * hsel.size();
    const size_t sh_off = sel_bytes + ((hfix.size() + 3) & ~(size_t)3);
    if (!binary) {
        gsel_.ensure(sh_off + hsh.size() * sizeof(uint32_t));
        CG_HIP(hipMemcpyAsync(gsel_.p, hsel.data(), sel_bytes, hipMemcpyHostToDevice, stream_));
        CG_HIP(hipMemcpyAsync(gsel_.as<uint8_t>() + sel_bytes, hfix.data(), hfix.size(), hipMemcpyHostToDevice,
                              stream_));
        CG_HIP(hipMemcpyAsync(gsel_.as<uint8_t>() + sh_off, hsh.data(), hsh.size() * sizeof(uint32_t),
                              hipMemcpyHostToDevice, stream_));
    }
    // incremental ranks when the digits they compute, plus the parent's
    // suffix sums (about two full ranks per state), stay under 90% of k
    // full ranks
    const uint8_t *d_gfix =
        (!binary && n >= 6 && k > 0 && 10 * (moved + 2 * (n - 2)) <= 9 * k * (n - 2) && !std::getenv("CG_RANK_FULL"))
            ? gsel_.as<uint8_t>() + sel_bytes
            : nullptr;

    // layer storage
    std::vector<uint64_t> off;  // keep_all: offsets of the layers in the arena
    uint64_t total = 1;         // states recorded so far
    if (keep_all) {
        // the whole orbit when it fits comfortably, else grow on demand
        size_t free_b = 0, total_b = 0;
        CG_HIP(hipMemGetInfo(&free_b, &total_b));
        uint64_t first = std::min<uint64_t>(spec.orbit_bound, 1ull << 20);
        if (spec.orbit_bound <= (uint64_t)(free_b / 4 / sizeof(uint64_t))) first = spec.orbit_bound;
        arena_.ensure(first * sizeof(uint64_t));
        CG_HIP(hipMemcpyAsync(arena_.p, &key0, 8, hipMemcpyHostToDevice, stream_));
        off.push_back(0);
        off.push_back(1);
    } else {
        lay_[0].ensure(64);  // L_{d-1} (empty at d = 0)
        lay_[1].ensure(64);
        CG_HIP(hipMemcpyAsync(lay_[1].p, &key0, 8, hipMemcpyHostToDevice, stream_));
    }
    int ip = 0, ic = 1, in = 2;  // indices of L_{d-1}, L_d, L_{d+1} in lay_
    uint64_t np = 0, F = 1;
    int iv = 0;          // directed: vis_[iv] holds every visited state, sorted
    uint64_t nvis = 0;
    if (directed) {
        vis_[0].ensure(64);
        CG_HIP(hipMemcpyAsync(vis_[0].p, &key0, 8, hipMemcpyHostToDevice, stream_));
        nvis = 1;
    }
    export_layer(spec, keep_all ? arena_.as<uint64_t>() : lay_[1].as<uint64_t>(), 1, written);

    // binary keys use bits [0, n); 4-bit keys [4, 4n) (the last entry of a
    // state follows from the others)
    const int bit_lo = binary ? 0 : 4, bit_hi = binary ? n : 4 * n;
    // Candidates sort as 32-bit lexicographic ranks when the states are
    // permutations of 0..n-1 with n <= 12 (12! < 2^32); layers stay packed.
    bool perm_start = !binary && n <= kRankMaxN;
    {
        bool seen[16] = {false};
        for (int i = 0; i < n && perm_start; ++i) {
            if (spec.start[i] >= n || seen[spec.start[i]]) perm_start = false;
            else seen[spec.start[i]] = true;
        }
    }
    const bool ranked = perm_start && !(spec.flags & CG_PACKED_SORT);
    // n = 13..16 with a permutation start: candidates sort as 64-bit ranks
    // (45 bits at n = 16: 6 passes of 8 bits instead of 8 over the 60 bits
    // of a packed key); reference layers are ranked as the dedup reads them
    bool perm_any = !binary && n > kRankMaxN;
    {
        bool seen[16] = {false};
        for (int i = 0; i < n && perm_any; ++i) {
            if (spec.start[i] >= n || seen[spec.start[i]]) perm_any = false;
            else seen[spec.start[i]] = true;
        }
    }
    const bool ranked64 = perm_any && !(spec.flags & CG_PACKED_SORT);
    // Ranked runs keep the ranks (32- or 64-bit) of layers d-1 and d beside
    // the packed layers (written by the gather), so the set difference does
    // not rank its reference keys again. A layer from the chunked path has
    // none; the next two steps then rank the packed layers on the fly.
    int kp = 0, kc = 1, kn = 2;
    bool rk_cur = false, rk_prev = false;
    if (ranked && !directed) {
        const uint32_t r0 = perm_rank(key0, n);
        rk_[kc].ensure(64);
        CG_HIP(hipMemcpyAsync(rk_[kc].p, &r0, sizeof r0, hipMemcpyHostToDevice, stream_));
        rk_cur = rk_prev = true;  // layer -1 is empty
    } else if (ranked64 && !directed) {
        uint64_t r0 = 0;
        with_rank64_n(n, [&](auto NN) { r0 = perm_rank_t<decltype(NN)::value, uint64_t>(key0); });
        rk_[kc].ensure(64);
        CG_HIP(hipMemcpyAsync(rk_[kc].p, &r0, sizeof r0, hipMemcpyHostToDevice, stream_));
        rk_cur = rk_prev = true;
    }
    int rank_bits = 0;
    while (rank_bits < 63 && (1ull << rank_bits) < spec.orbit_bound) ++rank_bits;
    int layers = 1;
    int status = CG_OK;
    for (;;) {
        if (k == 0) {
            status = CG_OK;
            break;
        }
        if (spec.max_frontier && F > spec.max_frontier) {
            status = CG_TRUNCATED;
            break;
        }
        if (layers >= spec.max_layers) {
            status = CG_TRUNCATED;
            break;
        }
        const uint64_t C = F * (uint64_t)k;
        const uint64_t room = spec.orbit_bound > total ? spec.orbit_bound - total : 0;
        const uint64_t out_cap = std::max<uint64_t>(1, std::min(C, room));
        const size_t key_bytes = ranked ? sizeof(uint32_t) : sizeof(uint64_t);
        // all candidates at once when both arrays fit; otherwise key-range
        // chunks sized to the memory left
        uint64_t cap = forced_chunk(C);
        if (cap >= C) {
            try {
                cand0_.ensure(C * key_bytes, 1.25);
                cand1_.ensure(C * key_bytes, 1.25);
            } catch (const Error &e) {
                if (e.code != CG_E_NOMEM) throw;
                cand0_.release();
                cand1_.release();
                cap = chunk_capacity(C, key_bytes);
            }
        }
        const bool chunked = cap < C;

        const uint64_t *Ld, *Lp;
        uint64_t *out;
        if (keep_all) {
            const uint64_t need = (total + out_cap) * sizeof(uint64_t);
            if (need > arena_.bytes) {
                // grow, keeping every layer (the arena holds them all)
                size_t want = std::max<size_t>(need, (size_t)(arena_.bytes * 1.5));
                want = std::min<size_t>(want, std::max<size_t>(need, spec.orbit_bound * 8));
                DevBuf bigger;
                bigger.stream = stream_;
                bigger.ensure(want);
                CG_HIP(hipMemcpyAsync(bigger.p, arena_.p, total * sizeof(uint64_t),
                                      hipMemcpyDeviceToDevice, stream_));
                CG_HIP(hipStreamSynchronize(stream_));
                arena_.swap(bigger);
            }
            const uint64_t d = off.size() - 2;  // index of L_d
            Ld = arena_.as<uint64_t>() + off[d];
            Lp = d > 0 ? arena_.as<uint64_t>() + off[d - 1] : nullptr;
            out = arena_.as<uint64_t>() + total;
        } else {
            Ld = lay_[ic].as<uint64_t>();
            Lp = lay_[ip].as<uint64_t>();
            out = nullptr;  // sized once N is known
        }

        // the states a candidate must not be: layers d and d-1, or (directed)
        // every visited state
        const uint64_t *Ra = directed ? vis_[iv].as<uint64_t>() : Ld;
        const uint64_t na = directed ? nvis : F;
        const uint64_t *Rb = directed ? nullptr : Lp;
        const uint64_t nb = directed ? 0 : np;
        uint64_t N = 0;
        bool rk_next = false;
        if (chunked) {
            uint64_t *dst = keep_all ? out : nullptr;
            N = run_chunked(ranked, n, Ld, F, Ra, na, Rb, nb, k, cap, rank_bits, bit_lo, bit_hi, dst, out_cap, room,
                            in);
            if (!keep_all) out = lay_[in].as<uint64_t>();
        } else if (ranked) {
            // candidates as 32-bit lexicographic ranks: half the bytes per
            // sort pass and only ceil(log2 n!) bits to sort
            uint32_t *c0 = cand0_.as<uint32_t>(), *c1 = cand1_.as<uint32_t>();
            const uint32_t *sorted = expand_rank_sort(n, Ld, F, gsel_.as<GenSel>(), d_gfix, k, c0, c1, rank_bits, w_);
            uint32_t *scratch = sorted == c0 ? c1 : c0;
            const bool by_rank = !directed && rk_cur && rk_prev;
            if (by_rank)
                launch_dedup_count_ranked_refs(n, sorted, C, rk_[kc].as<const uint32_t>(), F,
                                               rk_[kp].as<const uint32_t>(), np, scratch, w_.counter(), w_);
            else
                launch_dedup_count_ranked(n, sorted, C, Ra, na, Rb, nb, scratch, w_.counter(), w_);
            N = read_counter();
            if (N > C || N > room) throw Error(CG_E_DEVICE, "layer size out of range (device error)");
            if (!keep_all) {
                lay_[in].ensure(std::max<uint64_t>(N, 1) * sizeof(uint64_t), 1.25);
                out = lay_[in].as<uint64_t>();
            }
            uint32_t *rank_out = nullptr;
            if (!directed) {
                rk_[kn].ensure(std::max<uint64_t>(N, 1) * sizeof(uint32_t), 1.25);
                rank_out = rk_[kn].as<uint32_t>();
            }
            launch_dedup_gather_ranked(n, scratch, out, keep_all ? out_cap : N, w_, rank_out);
            rk_next = rank_out != nullptr;
        } else if (ranked64) {
            uint64_t *c0 = cand0_.as<uint64_t>(), *c1 = cand1_.as<uint64_t>();
            const uint64_t *sorted = expand_rank_sort64(n, Ld, F, gsel_.as<GenSel>(), k, c0, c1, rank_bits, w_);
            uint64_t *scratch = sorted == c0 ? c1 : c0;
            const bool by_rank = !directed && rk_cur && rk_prev;
            if (by_rank)
                launch_dedup_count_ranked64_refs(n, sorted, C, rk_[kc].as<const uint64_t>(), F,
                                                 rk_[kp].as<const uint64_t>(), np, scratch, w_.counter(), w_);
            else
                launch_dedup_count_ranked64(n, sorted, C, Ra, na, Rb, nb, scratch, w_.counter(), w_);
            N = read_counter();
            if (N > C || N > room) throw Error(CG_E_DEVICE, "layer size out of range (device error)");
            if (!keep_all) {
                lay_[in].ensure(std::max<uint64_t>(N, 1) * sizeof(uint64_t), 1.25);
                out = lay_[in].as<uint64_t>();
            }
            uint64_t *rank_out = nullptr;
            if (!directed) {
                rk_[kn].ensure(std::max<uint64_t>(N, 1) * sizeof(uint64_t), 1.25);
                rank_out = rk_[kn].as<uint64_t>();
            }
            launch_dedup_gather_ranked64(n, scratch, out, keep_all ? out_cap : N, w_, rank_out);
            rk_next = rank_out != nullptr;
        } else {
            const uint64_t *sorted;
            if (binary) {
                launch_expand_bits(Ld, F, gsel_.as<uint64_t>(), n, k, cand0_.as<uint64_t>(), w_);
                // the n key bits in balanced digits (38 bits: 7,7,8,8,8)
                sorted = radix_sort(cand0_.as<uint64_t>(), cand1_.as<uint64_t>(), C, bit_lo, bit_hi, w_, true);
            } else {
                sorted = expand_sort(Ld, F, gsel_.as<GenSel>(), k, cand0_.as<uint64_t>(), cand1_.as<uint64_t>(),
                                     bit_lo, bit_hi, w_);
            }
            uint64_t *scratch = sorted == cand0_.as<uint64_t>() ? cand1_.as<uint64_t>() : cand0_.as<uint64_t>();
            launch_dedup_count(sorted, C, Ra, na, Rb, nb, scratch, w_.counter(), w_);
            N = read_counter();
            if (N > C || N > room) throw Error(CG_E_DEVICE, "layer size out of range (device error)");
            if (!keep_all) {
                lay_[in].ensure(std::max<uint64_t>(N, 1) * sizeof(uint64_t), 1.25);
                out = lay_[in].as<uint64_t>();
            }
            launch_dedup_gather(scratch, out, keep_all ? out_cap : N, w_);
        }
        if (prof_.on) {
            prof_.collect();
            prof_.bytes[K_DEDUP] += 8.0 * (double)N;
        }
        res->states_expanded += F;
        res->candidates += C;
        if (N == 0) {
            status = CG_OK;
            break;
        }
        sizes[layers++] = N;
        export_layer(spec, out, N, written);
        total += N;
        if (directed) {
            // visited := visited merged with the new layer (disjoint, both sorted)
            vis_[iv ^ 1].ensure((nvis + N) * sizeof(uint64_t), 1.25);
            launch_merge(vis_[iv].as<uint64_t>(), nvis, out, N, vis_[iv ^ 1].as<uint64_t>(), stream_);
            iv ^= 1;
            nvis += N;
        }
        if (keep_all) {
            off.push_back(total);
        } else {
            const int t = ip;
            ip = ic;
            ic = in;
            in = t;
        }
        {
            const int t = kp;
            kp = kc;
            kc = kn;
            kn = t;
            rk_prev = rk_cur;
            rk_cur = rk_next;
        }
        np = F;
        F = N;
    }

    CG_HIP(hipEventRecord(ev1, stream_));
    CG_HIP(hipEventSynchronize(ev1));
    (void)read_counter();  // surfaces an error flag raised by the last gather
    float ms = 0;
    CG_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    prof_.collect();
    fill_kstats(prof_, res);
    res->device_ms = ms;
    res->status = status;
    res->num_layers = layers;
    const double t1 = now_seconds();
    res->t_submit = t0;
    res->t_admit = t0;
    res->t_done = t1;
}

}  // namespace cg
