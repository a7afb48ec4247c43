/*
 * cayleygrowth.h -- C ABI of libcayleygrowth.so: growth of permutation-group
 * Cayley graphs by layered breadth-first search on an MI355X (gfx950).
 *
 * What is computed (paper, section "Reminder on Cayley graphs, diameters,
 * growth", definition of Growth): for the graph whose vertices are the
 * states reachable from a start vector and whose edges join v and v.g for
 * every generator g, gamma(m) is the number of vertices at shortest-path
 * distance m from the start. The diameter (from the start) is the number of
 * layers minus one (same section). Generators are permutations in one-line
 * notation, 0-based (section "Examples and Tutorials"; explicit 0-based
 * definitions in section "Sheveleva2 and Koltsov3involutions").
 *
 * Action convention: gather, the neighbour t of state s under g has
 * t[i] = s[g[i]]. Layer SIZES do not depend on this choice; exported layer
 * CONTENTS do.
 *
 * Every call is exact integer work: layer counts are 64-bit and bit-exact.
 *
 * Threading: every entry point may be called from several host threads;
 * each call (or queue) owns its device buffers and stream. No C++
 * exception crosses this boundary.
 *
 * Memory: input pointers are host pointers borrowed for the duration of the
 * call (the queue copies what it needs before cg_queue_submit returns).
 * Output arrays are caller-owned host memory. Device memory is owned by the
 * library; it goes back to the library's device arena when a call returns
 * (queue: when a job retires) and to HIP (hipFree) on
 * cg_release_cached_memory().
 */
#ifndef CAYLEYGROWTH_H
#define CAYLEYGROWTH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define CG_OK 0            /* complete: an empty next layer was reached      */
#define CG_TRUNCATED 1     /* a stop rule ended the search (max_layers,
                              max_frontier); the last layer is non-empty     */
#define CG_PENDING 2       /* queue: the job has not finished yet            */
#define CG_E_INVAL (-1)    /* bad argument: n outside 1..16 (1..64 for
                              binary states), n_gens < 1, a generator row
                              that is not a permutation of 0..n-1,
                              max_layers < 1, NULL pointer, start entry > 15
                              (> 1 for binary states)                        */
#define CG_E_NOMEM (-2)    /* device or host memory exhausted                */
#define CG_E_DEVICE (-3)   /* HIP error or a kernel-reported failure         */
#define CG_E_UNSUPPORTED (-4) /* generating set not closed under inverses
                              and CG_ALLOW_DIRECTED not given                */
#define CG_E_BUSY (-5)     /* queue full, or workspace buffers in use         */
#define CG_E_CANCELLED (-6)/* job cancelled before it finished               */
#define CG_E_TIMEOUT (-7)  /* cg_queue_wait timed out (job still running)     */

/* ---- job flags ----------------------------------------------------------- */
#define CG_KEEP_ALL_LAYERS 0x1u  /* keep every layer resident on the device
                                    (otherwise only layers d-1, d, d+1)     */
#define CG_ALLOW_DIRECTED 0x2u   /* accept sets not closed under inverses;
                                    removes every earlier layer, not just
                                    d-1 and d (implies keeping all layers)  */
#define CG_START_STATE 0x4u      /* start from job.start instead of the
                                    identity (Schreier coset graphs: a start
                                    vector with repeated entries)            */
#define CG_PROFILE 0x8u          /* record per-kernel HIP-event timings into
                                    cg_result_t.kstats                        */
#define CG_PACKED_SORT 0x10u     /* sort candidates as packed 64-bit keys
                                    even when n <= 12 (by default they sort
                                    as 32-bit lexicographic ranks there)     */
#define CG_BITMASK 0x20u         /* run the bitmask engine instead of the
                                    sort-based one: three bitmaps over the
                                    n! lexicographic ranks (visited, layer d,
                                    layer d+1: 3 bits per state, the
                                    memory-saving encoding of the paper's
                                    section on growth benchmarks). n <= 14,
                                    start state a permutation, no layer
                                    export; n! * 3/8 bytes of device memory
                                    (32.7 GB at n = 14). Exact; directed
                                    sets allowed with CG_ALLOW_DIRECTED.     */
#define CG_SMALL_JOB 0x40u       /* run the whole job inside one workgroup
                                    (n <= 10, start a permutation, no layer
                                    export): one launch, rank-space bitmaps
                                    in LDS or a device slot; on a reusable
                                    engine the launch is a hipGraph that is
                                    replayed while the job's shape repeats */
#define CG_BINARY_STATE 0x80u    /* binary states: with CG_START_STATE and a
                                    0/1 start vector, pack one bit per entry
                                    instead of four (the Schreier coset
                                    graphs of the paper's section "Growth of
                                    Reversals and Transposons on binary
                                    cosets"). Implied for n > 16, up to
                                    n = 64. Sort path only (no CG_BITMASK,
                                    CG_SMALL_JOB, batches or queue); a
                                    layer's candidates must fit in device
                                    memory at once (no key-range chunks).   */

/*
 * A growth job.
 *   n            entries per state, 1..16 (each entry is packed in 4 bits);
 *                17..64 for binary states (CG_BINARY_STATE: 1 bit each)
 *   gens         n_gens rows of n bytes, row-major; row g holds the one-line
 *                images g[0..n-1]. Duplicate rows and the identity are
 *                allowed and ignored (they do not change any layer).
 *   n_gens       number of rows, >= 1
 *   max_layers   capacity of the caller's layer_sizes array, >= 1; at most
 *                this many layers (including layer 0) are computed
 *   max_frontier 0 = none; otherwise the first layer whose size is strictly
 *                greater than this is recorded and not expanded
 *   flags        CG_* job flags
 *   start        n bytes with entries 0..15 (0..1 for binary states) when
 *                CG_START_STATE is set, else ignored (NULL allowed)
 *   layers_out   optional host buffer (NULL = none): receives every
 *                recorded layer's states, layer after layer, each layer in
 *                increasing lexicographic order, n bytes per state
 *   layers_out_cap  capacity of layers_out in states; states beyond it are
 *                not written (the sizes still count them)
 */
typedef struct cg_job {
    int n;
    const uint8_t *gens;
    int n_gens;
    int max_layers;
    uint64_t max_frontier;
    uint32_t flags;
    const uint8_t *start;
    uint8_t *layers_out;
    uint64_t layers_out_cap;
} cg_job_t;

/* Per-kernel timing record (filled when CG_PROFILE is set). */
typedef struct cg_kstat {
    char name[32];
    uint64_t launches;
    double total_ms;   /* sum of HIP-event durations over all launches      */
    double alg_bytes;  /* algorithmic HBM bytes over all launches (what the
                          method itself must read and write)                */
    double items;      /* keys processed over all launches                   */
} cg_kstat_t;

#define CG_KSTAT_MAX 8

/*
 * Result of a job. layer_sizes is a caller-owned array of job.max_layers
 * entries; entries after the last recorded layer are set to 0.
 *   status          CG_OK, CG_TRUNCATED or a negative error code
 *   num_layers      recorded layers (diameter from the start = num_layers-1
 *                   when status == CG_OK)
 *   states_expanded sum of the sizes of the layers that were expanded
 *   candidates      neighbours generated (states_expanded x distinct gens)
 *   t_submit, t_admit, t_done   host monotonic seconds (queue jobs; the
 *                   plain calls set all three around the call)
 *   device_ms       HIP-event time from the first to the last kernel
 */
typedef struct cg_result {
    int status;
    int num_layers;
    uint64_t *layer_sizes;
    uint64_t states_expanded;
    uint64_t candidates;
    double t_submit, t_admit, t_done;
    double device_ms;
    int n_kstats;
    cg_kstat_t kstats[CG_KSTAT_MAX];
} cg_result_t;

/*
 * cg_growth -- growth from the identity (definition of Growth).
 * out_layer_sizes: caller-owned, max_layers entries, zero-filled after the
 * last layer. Returns CG_OK, CG_TRUNCATED, or a negative error. The set
 * must be closed under inverses (paper: the standard undirected case of the
 * section "Largest diameters found (and known) for n <= 15").
 */
int cg_growth(int n, const uint8_t *gens, int n_gens, int max_layers,
              uint64_t *out_layer_sizes);

/*
 * cg_growth_ex -- the full job interface. res->layer_sizes must point to
 * job->max_layers entries. stream: a hipStream_t to run on, or NULL for a
 * stream owned by the call. Returns res->status.
 */
int cg_growth_ex(const cg_job_t *job, cg_result_t *res, void *stream);

/*
 * A reusable engine: a stream plus device buffers kept between runs, so
 * that repeated jobs (benchmark steps, a worker serving many requests) do
 * not allocate per call. cg_engine_run has the semantics of cg_growth_ex.
 * One engine runs one job at a time; calls on one engine from several
 * threads are serialised by the caller. cg_engine_create returns NULL on
 * failure (see cg_last_error). cg_engine_destroy frees the buffers.
 */
typedef struct cg_engine cg_engine_t;
cg_engine_t *cg_engine_create(void *stream);
int cg_engine_run(cg_engine_t *eng, const cg_job_t *job, cg_result_t *res);
void cg_engine_destroy(cg_engine_t *eng);

/*
 * Batch options.
 *   stream         hipStream_t or NULL: the batch runs after the work already
 *                  queued on it (on a stream the library keeps per device,
 *                  so that its launch graph is replayed by later batches of
 *                  the same shape)
 *   max_active     most jobs advanced together in one tagged group (0 = auto)
 *   hbm_budget_bytes  reserved (the batch splits groups that run out of
 *                  device memory)
 *   tune           1 = let the autotuner choose, per size class (n), the
 *                  engine (one workgroup per job, or tagged groups), the
 *                  workgroup size and the jobs per group, and for the batch
 *                  the split that moves jobs far above their share of the
 *                  work to groups; choices are timed on the batch itself
 *                  and kept per device model in a file (CG_TUNE_CACHE, else
 *                  $XDG_CACHE_HOME or ~/.cache, cayleygrowth_tune.txt)
 */
typedef struct cg_batch_opts {
    void *stream;
    int max_active;
    uint64_t hbm_budget_bytes;
    int tune;
} cg_batch_opts_t;

/*
 * cg_growth_batch -- many independent jobs advanced together: their states
 * carry the job's index in the high key bits, so one expand, sort, unique,
 * set difference and compaction per super-step serves every active job.
 * Each result equals that job's cg_growth_ex result bit for bit. Workload
 * shape: the paper's searches over many generating sets (section "Largest
 * diameters found (and known) for n <= 15"). results[i].layer_sizes must
 * point to jobs[i].max_layers entries. opts may be NULL. Jobs must not set
 * CG_ALLOW_DIRECTED, CG_KEEP_ALL_LAYERS or layers_out (CG_E_INVAL).
 * Returns CG_OK when every job ran (see each results[i].status), or a
 * negative error for the whole batch.
 */
int cg_growth_batch(int n_jobs, const cg_job_t *jobs, cg_result_t *results,
                    const cg_batch_opts_t *opts);

/* What cg_growth_batch keeps on the current device between calls. */
typedef struct cg_batch_info {
    uint64_t calls;           /* cg_growth_batch calls on this device          */
    uint64_t graph_builds;    /* small-job launch graphs built                  */
    uint64_t graph_launches;  /* launches of such graphs (replays: launches
                                 minus builds)                                 */
    int tuned_classes;        /* size classes with autotuned choices           */
    double heavy_split;       /* tuned heavy-job split (1/x of the small-job
                                 work; 0 = not tuned)                          */
    int tune_file_entries;    /* choices read back from the tuning file        */
} cg_batch_info_t;

/* Fills *out for the current device. Returns CG_OK or CG_E_INVAL (NULL). */
int cg_batch_info(cg_batch_info_t *out);

/*
 * cg_growth_batch_noalloc -- cg_growth_batch for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc). It runs every job in the
 * small-job engine (one workgroup per job, one launch) and keeps all its
 * device buffers in one static array of the library (64 MiB, held by each
 * GPU the library runs on until the process ends): it calls no hipMalloc,
 * hipFree, event or stream creation. Results equal cg_growth_batch's bit
 * for bit.
 *   jobs, results  host arrays as for cg_growth_batch (inputs borrowed for
 *                  the call; results[i].layer_sizes caller-owned, holding
 *                  jobs[i].max_layers entries)
 *   stream         hipStream_t to run on, or NULL (the null stream); the
 *                  call synchronises it before returning
 * Limits (CG_E_INVAL beyond them, nothing launched): at most 4096 jobs;
 * every job with n <= 10, a permutation start and at most 128 distinct
 * generators (CG_ALLOW_DIRECTED allowed; no CG_KEEP_ALL_LAYERS or
 * layers_out); at most 32768 distinct generator rows and 2^21 recorded
 * layer sizes (sum over jobs of min(max_layers, n!)) in all. A job with a
 * bad generator row gets CG_E_INVAL in its own result. device_ms is the
 * host-timed span from the launch to the end of the read-back.
 * The array is shared by every call on one GPU and keeps the last call's
 * contents (the call clears what must start at zero). Calls that overlap
 * on one GPU would race on it; within this process they are serialised by
 * a lock per device.
 * Returns CG_OK when every job ran (see each results[i].status) or a
 * negative error for the whole call.
 */
int cg_growth_batch_noalloc(int n_jobs, const cg_job_t *jobs, cg_result_t *results, void *stream);

/* ---- serving: a request queue with continuous batching ------------------ */
typedef struct cg_queue cg_queue_t;

/*
 * Jobs with n <= 13 and orbits up to 2^21 states share one group of
 * job-tagged keys (continuous batching: they join and leave at super-step
 * boundaries); cheap jobs (n <= 10, n! * k <= 2^22) run in a small-job
 * lane, launch by launch. Larger jobs run on separate lanes (a thread, an
 * engine and a stream each), concurrently with the group.
 * Admission by device footprint: every admitted job is charged an upper
 * bound of the device bytes it can make the queue hold, and a job is
 * admitted only while the charges fit hbm_budget_bytes together. The one
 * exception: a job whose bound alone exceeds the budget is admitted when no
 * other job runs (it may then use more than the budget; its engine splits
 * layers into key-range chunks when device memory runs short). Lanes free
 * their device buffers when idle.
 *   hbm_budget_bytes  device bytes the active jobs may hold together
 *                     (0 = 60% of free memory at creation)
 *   max_active        most jobs in the shared group at once (0 = 256)
 *   max_queued        most jobs waiting (0 = 65536); beyond it CG_E_BUSY
 *   large_lanes       lanes for large jobs (0 = 2, at most 8)
 *   device            HIP device the queue runs on (-1 = the current one)
 *   stream            hipStream_t the shared group runs on (NULL = a stream
 *                     of its own); the lanes always use their own streams
 */
typedef struct cg_queue_opts {
    uint64_t hbm_budget_bytes;
    int max_active;
    int max_queued;
    int large_lanes;
    int device;
    void *stream;
} cg_queue_opts_t;

/* Queue statistics (cg_queue_stats). Bytes: charged = the admitted jobs'
   bounds; held = device bytes the queue's buffers hold, sampled after every
   super-step and job (peaks since creation); over_bound counts jobs,
   small-job launches and group super-steps that held more than they were
   charged (the shared group's fixed buffers, under 16 MiB, are not
   charged). */
typedef struct cg_queue_stats {
    uint64_t budget_bytes;
    uint64_t charged_bytes, peak_charged_bytes;
    uint64_t held_bytes, peak_held_bytes;
    int running, queued;
    uint64_t completed, cancelled, failed;
    uint64_t over_bound;
} cg_queue_stats_t;

/* Creates the queue and its engine thread; NULL on failure (cg_last_error). */
cg_queue_t *cg_queue_create(const cg_queue_opts_t *opts);

/*
 * Enqueue a job. The job's gens/start are copied before return; res_slot
 * and res_slot->layer_sizes must stay valid until the job is done,
 * cancelled or the queue is destroyed. *ticket receives the job's id.
 * Returns CG_OK, CG_E_INVAL or CG_E_BUSY.
 */
int cg_queue_submit(cg_queue_t *q, const cg_job_t *job, cg_result_t *res_slot,
                    uint64_t *ticket);

/* Once the job is done (res_slot filled): its status (CG_OK, CG_TRUNCATED
   or negative); before that CG_PENDING. CG_E_INVAL for an unknown ticket. */
int cg_queue_poll(cg_queue_t *q, uint64_t ticket);

/* Waits up to timeout_us (< 0 = forever). Returns like cg_queue_poll, or
   CG_E_TIMEOUT. A wait that returns the job's status releases the ticket
   (later calls with it return CG_E_INVAL). */
int cg_queue_wait(cg_queue_t *q, uint64_t ticket, int64_t timeout_us);

/* Cancels a queued or running job; it retires with CG_E_CANCELLED at the
   next super-step boundary (a job on the large-job lane that has started
   runs to completion). Returns CG_OK or CG_E_INVAL (unknown ticket). */
int cg_queue_cancel(cg_queue_t *q, uint64_t ticket);

/* Cancels what is left (queued jobs retire with CG_E_CANCELLED), drains the
   engine threads, frees everything. */
void cg_queue_destroy(cg_queue_t *q);

/* Fills *out with the queue's admission accounting and counters. Returns
   CG_OK or CG_E_INVAL (NULL argument). */
int cg_queue_stats(cg_queue_t *q, cg_queue_stats_t *out);

/*
 * Device memory: at its first large request the library reserves one
 * device arena (the fraction CG_ARENA_FRACTION of the free memory, default
 * 0.85; 0 disables it) and carves every buffer out of it; a freed range is
 * reused only after the work queued on its last stream has finished. This
 * frees the buffers and graphs that cg_growth_batch keeps between calls (a
 * batch call in progress finishes first; the next one builds them again),
 * then frees the arena (hipFree) if no buffer is in use (engines and
 * queues still alive keep theirs).
 */
void cg_release_cached_memory(void);

/*
 * Device memory of the library, for callers that size budgets or report
 * footprints (the paper's growth benchmarks state the memory a run needs).
 *   held_bytes       bytes its device buffers hold now (all devices;
 *                    engines, queues, batches, pipeline scratch)
 *   peak_held_bytes  the most they held at once since the last reset
 *   arena_bytes      device memory reserved as arenas (the buffers are
 *                    carved out of it; a caller's workspace not included)
 * The static array of cg_growth_batch_noalloc (64 MiB per device) is not
 * counted. reset_peak != 0 restarts the peak at the current value after
 * filling *out. Returns CG_OK or CG_E_INVAL (NULL out).
 */
typedef struct cg_memory_stats {
    uint64_t held_bytes;
    uint64_t peak_held_bytes;
    uint64_t arena_bytes;
} cg_memory_stats_t;
int cg_memory_stats(cg_memory_stats_t *out, int reset_peak);

/*
 * Hands the library device memory to carve its buffers from (for example a
 * tensor the caller allocated with PyTorch), on the current device:
 * dev_ptr..dev_ptr+bytes becomes the arena; requests it cannot hold fall
 * back to hipMalloc. The memory stays the caller's: the library never
 * frees it, and the caller must keep it alive until the workspace is
 * replaced. dev_ptr = NULL returns to an arena the library reserves itself.
 * The buffers that cg_growth_batch keeps between calls are freed first.
 * Returns CG_OK, CG_E_BUSY while buffers of engines or queues still live in
 * the current arena (destroy them first), or CG_E_INVAL (bytes too small,
 * under 64 KiB).
 */
int cg_set_workspace(void *dev_ptr, size_t bytes);

/* ---- growth statistics (host) -------------------------------------------- */
/*
 * The growth read as a distribution of the distance d from the start over
 * the reached states, p(d) = sizes[d] / total (paper, section "Table of
 * results: hundreds of new conjectures on Cayley graphs": mean, mode,
 * variance, skewness, kurtosis, and a Gaussian or Gumbel shape fitted to
 * the growth). Moments are population moments; kurtosis is the excess
 * kurtosis (m4 / var^2 - 3). The fits match moments: Gaussian (mean, sd);
 * Gumbel for the maximum when skewness >= 0, for the minimum otherwise,
 * with scale sd * sqrt(6) / pi and location mean -/+ 0.5772... * scale.
 * Each fit's distance is the total variation between p and the model's
 * mass on [d - 1/2, d + 1/2).
 */
typedef struct cg_growth_stats {
    uint64_t total;      /* states reached: sum of sizes                     */
    int diameter;        /* index of the last non-empty layer                */
    int mode;            /* first index of the largest layer                 */
    uint64_t max_layer;  /* size of that layer                               */
    uint64_t antipodes;  /* size of the last layer                           */
    double mean, variance, skewness, kurtosis;
    double gauss_mu, gauss_sigma, gauss_tv;
    double gumbel_mu, gumbel_beta, gumbel_tv;
    int gumbel_min;      /* 1: Gumbel of the minimum (left-skewed)          */
    int best_fit;        /* 0 Gaussian, 1 Gumbel (smaller distance)          */
} cg_growth_stats_t;

/* sizes: num_layers >= 1 layer sizes, host memory; trailing zeros ignored.
   Returns CG_OK, or CG_E_INVAL (NULL pointer, no layers, all zero). */
int cg_growth_stats(const uint64_t *sizes, int num_layers, cg_growth_stats_t *out);

/* ---- errors -------------------------------------------------------------- */
const char *cg_strerror(int code);
/* Detail string of the last failure on the calling thread ("" if none). */
const char *cg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CAYLEYGROWTH_H */
