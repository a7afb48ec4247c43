// Growth over rank-space bitmaps: a state of S_n is the bit at its
// lexicographic rank (a bijection onto [0, n!)), so a set of states is a
// bitmap of n! bits and membership is one bit test, exact by construction.
//
// Two engines share the per-candidate step (unrank, apply every generator,
// rank, test the visited bit, set the next-layer bit):
//   * the small-job engine runs one whole job per workgroup inside one
//     persistent launch; workgroups take jobs from a queue. Bitmaps live in
//     LDS for n <= 8 and in a per-workgroup slot of device memory for
//     n = 9, 10;
//   * the bitmask engine runs one large job over the whole device with
//     three bitmaps (visited, current layer, next layer: 3 bits per state,
//     the memory-saving encoding of the paper's section on growth
//     benchmarks), for n <= 14.
// Both keep a visited bitmap of every layer so far, so they are also
// correct for generating sets that are not closed under inverses.
#pragma once

#include <string>
#include <vector>

#include "engine.h"

namespace cg {

constexpr int kWgMaxN = 10;        // largest n of the small-job engine
constexpr int kBitmaskMaxN = 14;   // largest n of the bitmask engine
constexpr int kBitmapMaxK = 128;   // generators staged in LDS

// Start state is a permutation of 0..n-1 (rank space = S_n).
bool start_is_permutation(const JobSpec &spec);

// Launch shape of the small-job engine.
struct WgTuning {
    int block = 256;  // threads per workgroup
};

struct WgItem {
    const JobSpec *spec;
    cg_result_t *res;
};

// True when the job can run in the small-job engine.
bool wg_eligible(const JobSpec &spec);

// Device buffers of the small-job engine, reused across calls; the launch
// (queue reset + persistent kernel) is built once as a hipGraph (explicit
// kernel nodes) and replayed while its arguments stay the same.
class WgRunner {
public:
    explicit WgRunner(hipStream_t s);
    ~WgRunner();
    WgRunner(const WgRunner &) = delete;
    WgRunner &operator=(const WgRunner &) = delete;
    // Runs every item to completion and fills its result. Returns the
    // device time of the launch in ms.
    double run(std::vector<WgItem> &items, const WgTuning &t, double t_submit);
    // An upper bound of the device bytes one launch of `items` holds.
    static uint64_t launch_bytes(const std::vector<WgItem> &items, const WgTuning &t);
    // Device bytes the runner holds now; release() frees them.
    uint64_t device_bytes() const;
    void release();
    int graph_launches() const { return graph_launches_; }
    int graph_captures() const { return graph_captures_; }

private:
    hipStream_t stream_;
    DevBuf jobs_, gsel_, sizes_, outs_, ws_, ticket_;
    hipGraphExec_t exec_ = nullptr;
    hipGraph_t graph_ = nullptr;
    std::vector<uint64_t> graph_key_;
    int graph_launches_ = 0, graph_captures_ = 0;
};

// Picks the small-job workgroup size for jobs like `sample` by timing each
// candidate size on it with runner `r` (its device time to *best_ms_out).
WgTuning tune_wg(std::vector<WgItem> &sample, WgRunner &r, double *best_ms_out = nullptr);

// cg_growth_batch_noalloc: the small-job engine on the library's static
// device array (no allocation). Limits per call: jobs, distinct generator
// rows in all, and layer-size entries in all (sum of min(max_layers, n!)).
constexpr uint32_t kNoAllocMaxJobs = 4096;
constexpr uint32_t kNoAllocMaxGens = 32768;
constexpr uint64_t kNoAllocMaxSizes = 1ull << 21;
void run_batch_noalloc(int n_jobs, const cg_job_t *jobs, cg_result_t *results, hipStream_t stream);
// The current device's address of that array (taken once per device).
void *noalloc_scratch(int dev);

// The bitmask engine: whole-device growth of one job (n <= 14, start a
// permutation). Fills res like Engine::run. Layers are not exported.
void run_bitmask(const JobSpec &spec, cg_result_t *res, hipStream_t s);

// Why a job cannot use the bitmask engine ("" when it can).
std::string bitmask_unsupported(const JobSpec &spec);

}  // namespace cg
