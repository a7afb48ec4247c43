// Batched growth: many jobs advanced together in super-steps over
// job-tagged keys (see batch_kernels.hip for the key layout).
#pragma once

#include <vector>

#include "engine.h"

namespace cg {

// Per-job row of the device job table of one super-step.
struct BatchJobDev {
    uint64_t front_off;  // first index of the job's keys in the frontier
    uint64_t cand_off;   // first index of the job's candidates
    uint32_t kk;         // generators applied this step (0 = not expanded)
    uint32_t goff;       // first GenSel of the job in the table
};

void launch_batch_expand(const uint64_t *frontier, uint64_t total_f, const BatchJobDev *d_jobs,
                         const GenSel *d_gsel, uint64_t *out, int shift, uint64_t total_c,
                         uint32_t nslots, PipeWork &w);
// Per-slot key counts of a sorted batched layer (d_pos: nslots+1 scratch).
void launch_tag_count(const uint64_t *keys, uint64_t n, int shift, unsigned long long *d_cnt,
                      unsigned long long *d_pos, uint32_t nslots, PipeWork &w);
// out = merge of sorted a[0..na) and sorted b[0..nb) (no key in both).
void launch_merge(const uint64_t *a, uint64_t na, const uint64_t *b, uint64_t nb, uint64_t *out,
                  hipStream_t s);

// State of one job inside a group.
struct SlotJob {
    JobSpec spec;
    cg_result_t *res = nullptr;  // caller's result (layer_sizes filled in place)
    uint64_t F = 0;              // current layer size
    int layers = 1;
    bool done = false;
    int status = CG_OK;
    double t_submit = 0, t_admit = 0;
    uint32_t goff = 0;           // first GenSel in the group table
    uint64_t key0 = 0;           // tagged start key
};

// A group of jobs sharing super-steps on one engine's stream and buffers.
// Jobs may join at a super-step boundary into free slots; a slot is reused
// only after its previous job's keys left layers d and d-1 (two steps).
class BatchGroup {
public:
    BatchGroup(hipStream_t stream, int n_max, int slots);
    ~BatchGroup();
    int capacity() const { return (int)slot_.size(); }
    int shift() const { return shift_; }
    int n_max() const { return n_max_; }
    // A free slot, or -1.
    int free_slot() const;
    // Adds a job (spec.n <= n_max) into `slot` before the next step.
    void add(int slot, const JobSpec &spec, cg_result_t *res, double t_submit, double t_admit);
    // True when no job is running.
    bool idle() const;
    // One super-step for every running job. Jobs that finish have their
    // result written and are returned in `finished`.
    void step(std::vector<int> &finished);
    // Cancels the job in `slot` (retires with CG_E_CANCELLED).
    void cancel(int slot);
    bool occupied(int slot) const { return slot >= 0 && slot < (int)slot_.size() && slot_[slot].res; }
    uint64_t device_bytes() const;
    // With no job running: drops the keys finished jobs left in the layer
    // windows (their slots become free at once) and frees the large
    // buffers. Returns false (and does nothing) while a job runs.
    bool release_idle();

private:
    void finish(int slot, int status);
    void rebuild_gensel();

    hipStream_t stream_;
    int n_max_, shift_, tag_bits_;
    std::vector<SlotJob> slot_;
    std::vector<int> quarantine_;  // steps until a freed slot may be reused
    std::vector<uint64_t> pending_keys_;  // tagged start keys of jobs joining
    std::vector<GenSel> hsel_;
    bool sel_dirty_ = true;
    PipeWork w_;
    DevBuf gsel_, jobs_, cand0_, cand1_, lay_[3], cnt_, pos_, join_, merged_;
    int ip_ = 0, ic_ = 1, in_ = 2;
    uint64_t nprev_ = 0, ncur_ = 0;  // sizes of layers d-1 and d (all jobs)
    uint64_t *host_ = nullptr;       // pinned: per-slot counts + flags
    size_t host_cap_ = 0;
};

// cg_growth_batch: groups by n (a size class), at most 2^tag_bits jobs each.
void run_batch(int n_jobs, const cg_job_t *jobs, cg_result_t *results, const cg_batch_opts_t *opts);
// cg_batch_info for the current device.
void batch_info(cg_batch_info_t *out);
// Frees the device buffers and graphs that batches keep between calls (on
// every device; the next batch builds them again).
void release_batch_buffers();

}  // namespace cg
