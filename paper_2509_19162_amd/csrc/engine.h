// Single-job growth engine: the layer loop of the breadth-first search.
#pragma once

#include <vector>

#include "../../include/cayleygrowth.h"
#include "internal.h"

namespace cg {

// A validated job (generators deduplicated, identity dropped).
struct JobSpec {
    int n = 0;
    int k = 0;                  // distinct non-identity generators
    std::vector<uint8_t> gens;  // k rows of n bytes
    bool inverse_closed = true;
    bool binary = false;        // one bit per entry (0/1 start vector, n <= 64)
    uint8_t start[64] = {0};
    int max_layers = 1;
    uint64_t max_frontier = 0;
    uint32_t flags = 0;
    uint8_t *layers_out = nullptr;
    uint64_t layers_out_cap = 0;
    uint64_t orbit_bound = 1;  // n! / prod(mult!) of the start's entries
};

// Validates and canonicalises a job; throws Error(CG_E_INVAL / _UNSUPPORTED).
JobSpec canonicalize(const cg_job_t &job, bool batch);

double now_seconds();

// Sets the calling thread's cg_last_error() string.
void set_last_error(const std::string &msg);

class Engine {
public:
    explicit Engine(hipStream_t user_stream);
    ~Engine();
    Engine(const Engine &) = delete;
    Engine &operator=(const Engine &) = delete;

    // Runs the job to completion; fills res (layer_sizes must hold
    // spec.max_layers entries). Throws Error on failure.
    void run(const JobSpec &spec, cg_result_t *res);

    PipeWork &work() { return w_; }
    hipStream_t stream() const { return stream_; }
    // Reads back one u64 counter and the kernel error flag (synchronises).
    uint64_t read_counter();
    // Device bytes the engine's buffers hold now (they are kept between
    // runs); release_buffers() frees them.
    uint64_t device_bytes() const;
    void release_buffers();

private:
    void export_layer(const JobSpec &spec, const uint64_t *d_keys, uint64_t count,
                      uint64_t &written);
    uint64_t forced_chunk(uint64_t C);
    uint64_t chunk_capacity(uint64_t C, size_t key_bytes);
    bool binary_ = false;  // the current run's states are binary (one bit per entry)
    uint64_t run_chunked(bool ranked, int n, const uint64_t *Ld, uint64_t F, const uint64_t *Ra, uint64_t na,
                         const uint64_t *Rb, uint64_t nb, int k, uint64_t cap, int rank_bits, int bit_lo, int bit_hi,
                         uint64_t *dst, uint64_t out_cap, uint64_t room, int in);

    hipStream_t stream_ = nullptr;
    bool own_stream_ = false;
    PipeWork w_;
    Profiler prof_;
    DevBuf gsel_, cand0_, cand1_, lay_[3], arena_, stage_, chunk_hist_, vis_[2];
    DevBuf rk_[3];  // ranked runs: 32-bit ranks of layers d-1, d, d+1
    class WgRunner *wg_ = nullptr;  // small-job engine (created on first use)
    static constexpr size_t kHostSmallBytes = 512;
    uint64_t *host_small_ = nullptr;  // pinned: error flag .. counter
};

void fill_kstats(const Profiler &p, cg_result_t *res);

}  // namespace cg
