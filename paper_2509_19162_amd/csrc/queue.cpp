// Serving: a request queue with continuous batching (cg_queue_*).
//
// Cheap jobs (a permutation start, n! * k <= 2^22 candidates) go to a
// small-job lane: each launch of the one-workgroup-per-job engine takes
// the cheap jobs queued at that moment (as many as the budget allows), and
// jobs that arrive meanwhile join the next launch.
//
// Client threads submit growth jobs; an engine thread admits queued jobs
// into free slots of a shared group (job-tagged keys, see
// batch_kernels.hip) at a super-step boundary, runs one super-step for
// every admitted job, and retires finished jobs (result written,
// timestamps set, waiters woken). Large jobs (n > 13, an orbit above 2^21
// states, or a bound above a quarter of the budget) run on separate lanes,
// each a thread with its own engine and stream, so their work overlaps with
// the shared group's on the device and they do not hold back the small
// jobs' super-steps; from n = 12 such permutation jobs use the bitmask
// engine.
//
// Device memory: every admitted request is charged an upper bound of the
// device bytes it can make the queue hold (job_bound below; for a
// small-job launch, the launch's buffers), and every lane admits only while
// the charges fit the budget together. The one exception keeps the queue
// moving: a request whose bound alone exceeds the budget is admitted when
// nothing else runs. Lanes free their buffers when they go idle, so what
// the queue holds never exceeds what it has charged.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "batch.h"
#include "bitmap.h"

namespace cg {

namespace {

constexpr int kSharedN = 13;  // 4*13 state bits + 12 tag bits = 64
constexpr uint64_t kSmallLaneWork = 1ull << 22;  // n! * k candidates at most
constexpr uint64_t kLargeOrbit = 1ull << 21;

uint64_t factorial_u64(int n) {
    uint64_t f = 1;
    for (int i = 2; i <= n; ++i) f *= (uint64_t)i;
    return f;
}

// Upper bound of the device bytes one job can make an engine or a group
// hold. Sort path, per candidate: two key arrays (8 B each), look-back words
// (at most 0.5 B), kill flags (1 B); per state of a layer: three packed
// windows (8 B) and their ranks (up to 8 B); directed sets: the sorted visited
// array twice (8 B per state). A layer holds at most min(orbit, k * F)
// states and an expanded one at most min(orbit, max_frontier), so the
// candidates of one step are at most k * F. Buffers may grow with 50%
// slack; 64 MiB covers the fixed ones. Bitmask engine: its three bitmaps
// and their summaries, exactly.
uint64_t job_bound(const JobSpec &s) {
    const double k = (double)std::max(1, s.k);
    const double orbit = (double)s.orbit_bound;
    if (s.flags & CG_BITMASK) {
        const double words = std::ceil((double)factorial_u64(s.n) / 32.0);
        return (uint64_t)(12.0 * words + 8.0 * std::ceil(words / 1024.0 / 32.0)) + (64ull << 20);
    }
    double F = orbit;
    if (s.max_frontier) F = std::min(F, (double)s.max_frontier);
    const double L = std::min(orbit, k * F);
    double b = k * F * 17.5 + 3.0 * 16.0 * L;
    if (!s.inverse_closed) b += 16.0 * orbit;
    return (uint64_t)(1.5 * b) + (64ull << 20);
}

}  // namespace

struct QueueReq {
    uint64_t ticket = 0;
    JobSpec spec;
    cg_result_t *res = nullptr;
    double t_submit = 0;
    int state = 0;  // 0 queued, 1 running, 2 done
    int status = CG_PENDING;
    bool cancel = false;
    bool big = false;
    int slot = -1;
    uint64_t bound = 0;   // job_bound(spec): what admission charges it
    uint64_t charged = 0; // charged now (0 until admitted; a small-job launch
                          // charges its whole launch to its first job)
};

}  // namespace cg

struct cg_queue {
    cg_queue_opts_t opts{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread engine;
    std::thread small_lane;
    std::vector<std::thread> big_lanes;
    bool stopping = false;
    uint64_t next_ticket = 1;
    uint64_t budget = 0;
    // admission accounting (all under mu)
    uint64_t in_use = 0, peak_in_use = 0;  // charged bytes
    int running = 0;                       // admitted, not yet retired
    std::vector<uint64_t> held;            // bytes each lane holds (0: group, 1: small, 2..: large)
    uint64_t peak_held = 0;
    uint64_t completed = 0, cancelled = 0, failed = 0;
    uint64_t over_bound = 0;  // a job, launch or group step held more than it was charged
    std::deque<cg::QueueReq *> queued, big_queued, small_queued;
    std::map<uint64_t, std::unique_ptr<cg::QueueReq>> reqs;
    std::string fatal;  // non-empty once the engine failed

    void engine_loop();
    void big_loop(int lane);
    void small_loop();
    // caller holds mu for all of these
    bool fits(uint64_t bytes) const { return running == 0 || in_use + bytes <= budget; }
    void charge(cg::QueueReq *r, uint64_t bytes);
    void retire(cg::QueueReq *r, int status);
    void set_held(size_t lane, uint64_t bytes);
};

void cg_queue::charge(cg::QueueReq *r, uint64_t bytes) {
    r->charged = bytes;
    r->state = 1;
    in_use += bytes;
    ++running;
    peak_in_use = std::max(peak_in_use, in_use);
}

void cg_queue::retire(cg::QueueReq *r, int status) {
    // a request that was never admitted holds no charge
    if (r->state == 1) {
        in_use -= std::min(in_use, r->charged);
        --running;
    }
    r->charged = 0;
    r->state = 2;
    r->status = status;
    r->res->status = status;
    if (status == CG_E_CANCELLED)
        ++cancelled;
    else if (status < 0)
        ++failed;
    else
        ++completed;
    cv_done.notify_all();
    cv_work.notify_all();  // charges freed: other lanes may admit
}

void cg_queue::set_held(size_t lane, uint64_t bytes) {
    if (lane >= held.size()) return;
    held[lane] = bytes;
    uint64_t sum = 0;
    for (uint64_t b : held) sum += b;
    peak_held = std::max(peak_held, sum);
}

namespace {

// A request that is retired without having run.
void stamp_unrun(cg::QueueReq *r) {
    r->res->t_submit = r->t_submit;
    r->res->t_admit = r->res->t_done = cg::now_seconds();
    r->res->num_layers = 0;
}

}  // namespace

void cg_queue::engine_loop() {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::unique_ptr<cg::BatchGroup> group;
    std::map<int, cg::QueueReq *> by_slot;
    try {
        CG_HIP(hipSetDevice(device));
        if (opts.stream) {
            stream = (hipStream_t)opts.stream;
        } else {
            CG_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
            own_stream = true;
        }
        const int cap = std::max(1, std::min(opts.max_active > 0 ? opts.max_active : 256, 4096));
        group.reset(new cg::BatchGroup(stream, cg::kSharedN, cap));
        // the group's fixed buffers (slot tables, pipeline counters) are not
        // charged: they stay small and exist for the queue's lifetime
        const uint64_t group_base = group->device_bytes() + (16ull << 20);
        std::vector<int> fin;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] {
                    return stopping || !group->idle() ||
                           (!queued.empty() && (queued.front()->cancel || fits(queued.front()->bound)));
                });
                if (stopping && group->idle()) {
                    // requests still waiting are cancelled
                    for (auto *r : queued) {
                        stamp_unrun(r);
                        retire(r, CG_E_CANCELLED);
                    }
                    queued.clear();
                    break;
                }
                // cancellations take effect at this super-step boundary
                for (auto it = by_slot.begin(); it != by_slot.end();) {
                    if (it->second->cancel || stopping) {
                        group->cancel(it->first);
                        cg::QueueReq *r = it->second;
                        r->res->t_done = cg::now_seconds();
                        retire(r, CG_E_CANCELLED);
                        it = by_slot.erase(it);
                    } else {
                        ++it;
                    }
                }
                // admission: FIFO while a slot and the budget allow
                while (!stopping && !queued.empty()) {
                    cg::QueueReq *r = queued.front();
                    if (r->cancel) {
                        queued.pop_front();
                        stamp_unrun(r);
                        retire(r, CG_E_CANCELLED);
                        continue;
                    }
                    const int slot = group->free_slot();
                    if (slot < 0 || !fits(r->bound)) break;
                    queued.pop_front();
                    charge(r, r->bound);
                    r->slot = slot;
                    group->add(slot, r->spec, r->res, r->t_submit, cg::now_seconds());
                    by_slot[slot] = r;
                }
            }
            if (!group->idle()) group->step(fin);
            const uint64_t held_step = group->device_bytes();  // buffers only grow within a step
            (void)group->release_idle();  // frees the buffers once no job runs
            const uint64_t held_now = group->device_bytes();
            std::lock_guard<std::mutex> lk(mu);
            uint64_t charged = group_base;
            for (auto &kv : by_slot) charged += kv.second->charged;
            if (held_step > charged) ++over_bound;
            set_held(0, held_step);
            set_held(0, held_now);
            for (int s : fin) {
                auto it = by_slot.find(s);
                if (it == by_slot.end()) continue;
                retire(it->second, it->second->res->status);
                by_slot.erase(it);
            }
        }
    } catch (const std::exception &e) {
        std::lock_guard<std::mutex> lk(mu);
        fatal = e.what();
        for (auto &kv : by_slot) retire(kv.second, CG_E_DEVICE);
        for (auto *r : queued) {
            stamp_unrun(r);
            retire(r, CG_E_DEVICE);
        }
        queued.clear();
    }
    group.reset();
    {
        std::lock_guard<std::mutex> lk(mu);
        set_held(0, 0);
    }
    if (stream) {
        (void)hipStreamSynchronize(stream);
        if (own_stream) (void)hipStreamDestroy(stream);
    }
}

void cg_queue::big_loop(int lane) {
    std::unique_ptr<cg::Engine> eng;
    const size_t slot = 2 + (size_t)lane;
    (void)hipSetDevice(device);
    for (;;) {
        cg::QueueReq *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            // admission: the head of the large-job queue starts when its
            // bound fits beside everything charged so far
            cv_work.wait(lk, [&] {
                return stopping || (!big_queued.empty() &&
                                    (big_queued.front()->cancel || fits(big_queued.front()->bound)));
            });
            if (big_queued.empty()) break;
            r = big_queued.front();
            big_queued.pop_front();
            if (r->cancel || stopping) {
                stamp_unrun(r);
                retire(r, CG_E_CANCELLED);
                continue;
            }
            charge(r, r->bound);
        }
        const double t_admit = cg::now_seconds();
        int status;
        uint64_t held_end = 0;
        try {
            if (!eng) eng.reset(new cg::Engine(nullptr));
            eng->run(r->spec, r->res);
            status = r->res->status;
            held_end = eng->device_bytes();  // buffers only grow during a run
            eng->release_buffers();
        } catch (const cg::Error &e) {
            status = e.code;
            eng.reset();  // frees whatever the failed run held
        } catch (...) {
            status = CG_E_DEVICE;
            eng.reset();
        }
        std::lock_guard<std::mutex> lk(mu);
        if (held_end > r->charged) ++over_bound;
        set_held(slot, held_end);
        set_held(slot, eng ? eng->device_bytes() : 0);
        r->res->t_submit = r->t_submit;
        r->res->t_admit = t_admit;
        r->res->t_done = cg::now_seconds();
        retire(r, status);
    }
}

// Small jobs (n <= 10, a permutation start): each launch of the small-job
// engine runs the small jobs queued at that moment, one workgroup per job,
// as many as the budget allows beside what is charged already; jobs that
// arrive meanwhile join the next launch. A job that has started runs to
// completion (a cancel then has no effect).
void cg_queue::small_loop() {
    hipStream_t stream = nullptr;
    std::unique_ptr<cg::WgRunner> runner;
    const cg::WgTuning tuning;
    try {
        CG_HIP(hipSetDevice(device));
        CG_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
        runner.reset(new cg::WgRunner(stream));
        for (;;) {
            std::vector<cg::QueueReq *> batch;
            std::vector<cg::WgItem> items;
            {
                std::unique_lock<std::mutex> lk(mu);
                auto head_fits = [&] {
                    if (small_queued.empty()) return false;
                    cg::QueueReq *h = small_queued.front();
                    if (h->cancel) return true;
                    std::vector<cg::WgItem> one{{&h->spec, h->res}};
                    return fits(cg::WgRunner::launch_bytes(one, tuning));
                };
                cv_work.wait(lk, [&] { return stopping || head_fits(); });
                if (small_queued.empty()) break;
                uint64_t bytes = 0;
                while (!small_queued.empty()) {
                    cg::QueueReq *r = small_queued.front();
                    if (r->cancel || stopping) {
                        small_queued.pop_front();
                        stamp_unrun(r);
                        retire(r, CG_E_CANCELLED);
                        continue;
                    }
                    items.push_back({&r->spec, r->res});
                    const uint64_t b = cg::WgRunner::launch_bytes(items, tuning);
                    if (!batch.empty() && !(in_use + b <= budget)) {
                        items.pop_back();
                        break;
                    }
                    if (batch.empty() && !fits(b)) {
                        items.pop_back();
                        break;
                    }
                    small_queued.pop_front();
                    batch.push_back(r);
                    bytes = b;
                }
                if (batch.empty()) continue;
                // the launch's bytes are charged to its first job; the
                // others run under that charge
                charge(batch[0], bytes);
                for (size_t i = 1; i < batch.size(); ++i) charge(batch[i], 0);
            }
            int status = CG_OK;
            uint64_t held_end = 0;
            try {
                runner->run(items, tuning, 0.0);
                held_end = runner->device_bytes();
                runner->release();
            } catch (const cg::Error &e) {
                status = e.code;
                runner->release();
            }
            std::lock_guard<std::mutex> lk(mu);
            if (held_end > batch[0]->charged) ++over_bound;
            set_held(1, held_end);
            set_held(1, 0);
            for (auto *r : batch) {
                r->res->t_submit = r->t_submit;
                retire(r, status == CG_OK ? r->res->status : status);
            }
        }
    } catch (const std::exception &e) {
        std::lock_guard<std::mutex> lk(mu);
        fatal = e.what();
        for (auto *r : small_queued) {
            stamp_unrun(r);
            retire(r, CG_E_DEVICE);
        }
        small_queued.clear();
    }
    runner.reset();
    if (stream) {
        (void)hipStreamSynchronize(stream);
        (void)hipStreamDestroy(stream);
    }
}

extern "C" {

cg_queue_t *cg_queue_create(const cg_queue_opts_t *opts) {
    try {
        std::unique_ptr<cg_queue> q(new cg_queue());
        if (opts)
            q->opts = *opts;
        else
            q->opts.device = -1;
        if (q->opts.device >= 0) {
            int count = 0;
            CG_HIP(hipGetDeviceCount(&count));
            if (q->opts.device >= count) throw cg::Error(CG_E_INVAL, "queue device out of range");
            q->device = q->opts.device;
        } else {
            CG_HIP(hipGetDevice(&q->device));
        }
        int prev = 0;
        CG_HIP(hipGetDevice(&prev));
        CG_HIP(hipSetDevice(q->device));
        size_t free_b = 0, total_b = 0;
        const hipError_t e = hipMemGetInfo(&free_b, &total_b);
        (void)hipSetDevice(prev);
        CG_HIP(e);
        q->budget = q->opts.hbm_budget_bytes ? q->opts.hbm_budget_bytes : (uint64_t)(0.6 * (double)free_b);
        const int lanes = q->opts.large_lanes > 0 ? std::min(q->opts.large_lanes, 8) : 2;
        q->held.assign(2 + (size_t)lanes, 0);
        q->engine = std::thread([p = q.get()] { p->engine_loop(); });
        q->small_lane = std::thread([p = q.get()] { p->small_loop(); });
        for (int i = 0; i < lanes; ++i) q->big_lanes.emplace_back([p = q.get(), i] { p->big_loop(i); });
        return q.release();
    } catch (const std::exception &e) {
        cg::set_last_error(e.what());
        return nullptr;
    }
}

int cg_queue_submit(cg_queue_t *q, const cg_job_t *job, cg_result_t *res_slot, uint64_t *ticket) {
    if (!q || !job || !res_slot || !res_slot->layer_sizes || !ticket) return CG_E_INVAL;
    std::unique_ptr<cg::QueueReq> r(new cg::QueueReq());
    try {
        r->spec = cg::canonicalize(*job, true);  // copies gens and start
    } catch (const cg::Error &e) {
        cg::set_last_error(e.what());
        return e.code;
    }
    r->res = res_slot;
    r->t_submit = cg::now_seconds();
    r->bound = cg::job_bound(r->spec);
    res_slot->status = CG_PENDING;
    std::lock_guard<std::mutex> lk(q->mu);
    if (!q->fatal.empty() || q->stopping) return CG_E_DEVICE;
    const int max_q = q->opts.max_queued > 0 ? q->opts.max_queued : 65536;
    if ((int)(q->queued.size() + q->big_queued.size() + q->small_queued.size()) >= max_q) return CG_E_BUSY;
    r->ticket = q->next_ticket++;
    // cheap jobs only: one workgroup runs the whole job, and a launch lasts
    // as long as its slowest job
    const uint64_t states = cg::factorial_u64(r->spec.n);
    const bool small = r->spec.n <= cg::kWgMaxN && cg::wg_eligible(r->spec) &&
                       states * (uint64_t)std::max(1, r->spec.k) <= cg::kSmallLaneWork;
    // the shared group subtracts layers d and d-1 only: directed jobs that
    // are not small take a lane (its engine subtracts every visited state)
    r->big = !small && (!r->spec.inverse_closed || r->spec.n > cg::kSharedN ||
                        r->spec.orbit_bound > cg::kLargeOrbit || r->bound > q->budget / 4);
    // large permutation jobs from n = 12 run in the bitmask engine: 3 bits
    // per state of S_n instead of 8-byte layers and candidate arrays (an
    // S_13 job holds 2.3 GB there); results are the same
    if (r->big && r->spec.n >= 12 && !(r->spec.flags & CG_PACKED_SORT) && cg::bitmask_unsupported(r->spec).empty()) {
        r->spec.flags |= CG_BITMASK;
        r->bound = cg::job_bound(r->spec);
    }
    *ticket = r->ticket;
    cg::QueueReq *p = r.get();
    q->reqs[r->ticket] = std::move(r);
    if (p->big) {
        q->big_queued.push_back(p);
    } else if (small) {
        q->small_queued.push_back(p);
    } else {
        q->queued.push_back(p);
    }
    q->cv_work.notify_all();
    return CG_OK;
}

int cg_queue_poll(cg_queue_t *q, uint64_t ticket) {
    if (!q) return CG_E_INVAL;
    std::lock_guard<std::mutex> lk(q->mu);
    auto it = q->reqs.find(ticket);
    if (it == q->reqs.end()) return CG_E_INVAL;
    return it->second->state == 2 ? it->second->status : CG_PENDING;
}

int cg_queue_wait(cg_queue_t *q, uint64_t ticket, int64_t timeout_us) {
    if (!q) return CG_E_INVAL;
    std::unique_lock<std::mutex> lk(q->mu);
    auto it = q->reqs.find(ticket);
    if (it == q->reqs.end()) return CG_E_INVAL;
    cg::QueueReq *r = it->second.get();
    auto done = [&] { return r->state == 2; };
    if (timeout_us < 0) {
        q->cv_done.wait(lk, done);
    } else if (!q->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done)) {
        return CG_E_TIMEOUT;
    }
    const int status = r->status;
    q->reqs.erase(ticket);  // a finished wait releases the ticket
    return status;
}

int cg_queue_cancel(cg_queue_t *q, uint64_t ticket) {
    if (!q) return CG_E_INVAL;
    std::lock_guard<std::mutex> lk(q->mu);
    auto it = q->reqs.find(ticket);
    if (it == q->reqs.end()) return CG_E_INVAL;
    it->second->cancel = true;
    q->cv_work.notify_all();
    return CG_OK;
}

int cg_queue_stats(cg_queue_t *q, cg_queue_stats_t *out) {
    if (!q || !out) return CG_E_INVAL;
    std::lock_guard<std::mutex> lk(q->mu);
    std::memset(out, 0, sizeof *out);
    out->budget_bytes = q->budget;
    out->charged_bytes = q->in_use;
    out->peak_charged_bytes = q->peak_in_use;
    uint64_t held = 0;
    for (uint64_t b : q->held) held += b;
    out->held_bytes = held;
    out->peak_held_bytes = q->peak_held;
    out->running = q->running;
    out->queued = (int)(q->queued.size() + q->big_queued.size() + q->small_queued.size());
    out->completed = q->completed;
    out->cancelled = q->cancelled;
    out->failed = q->failed;
    out->over_bound = q->over_bound;
    return CG_OK;
}

void cg_queue_destroy(cg_queue_t *q) {
    if (!q) return;
    {
        std::lock_guard<std::mutex> lk(q->mu);
        q->stopping = true;
        q->cv_work.notify_all();
    }
    if (q->engine.joinable()) q->engine.join();
    if (q->small_lane.joinable()) q->small_lane.join();
    for (auto &t : q->big_lanes)
        if (t.joinable()) t.join();
    delete q;
}

}  // extern "C"
