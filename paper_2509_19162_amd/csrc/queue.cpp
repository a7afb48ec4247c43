// Serving: a request queue with continuous batching (cg_queue_*).
//
// Cheap jobs (a permutation start, n! * k <= 2^22 candidates) go to a
// small-job lane: each launch of the one-workgroup-per-job engine takes
// every such job queued at that moment, and jobs that arrive meanwhile
// join the next launch.
//
// Client threads submit growth jobs; an engine thread admits queued jobs
// while their estimated device footprint fits the budget, adds them into
// free slots of a shared group (job-tagged keys, see batch_kernels.hip) at
// a super-step boundary, runs one super-step for every admitted job, and
// retires finished jobs (result written, timestamps set, waiters woken).
// Large jobs (n > 13, an orbit above 2^21 states, or an estimate above a
// quarter of the budget) run on separate lanes, each a thread with its own
// engine and stream, so their work overlaps with the shared group's on the
// device and they do not hold back the small jobs' super-steps; from n = 12
// such permutation jobs use the bitmask engine.
#include <algorithm>
#include <atomic>
#include <chrono>
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

// Upper estimate of a job's peak device bytes: the largest layer is taken
// as 35% of the orbit (capped by what the stop rules allow), times the
// three layer windows and two candidate buffers with 25% slack.
uint64_t estimate_bytes(const JobSpec &s) {
    double layer = 0.35 * (double)s.orbit_bound;
    if (s.max_frontier) layer = std::min(layer, (double)s.max_frontier * std::max(1, s.k));
    if (layer < 1) layer = 1;
    return (uint64_t)(8.0 * layer * (3.0 + 2.5 * std::max(1, s.k))) + (1u << 20);
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
    uint64_t bytes = 0;
};

}  // namespace cg

struct cg_queue {
    cg_queue_opts_t opts{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread engine;
    std::thread small_lane;
    std::vector<std::thread> big_lanes;
    int big_running = 0;
    bool stopping = false;
    uint64_t next_ticket = 1;
    uint64_t budget = 0, in_use = 0;
    std::deque<cg::QueueReq *> queued, big_queued, small_queued;
    std::map<uint64_t, std::unique_ptr<cg::QueueReq>> reqs;
    std::string fatal;  // non-empty once the engine failed

    void engine_loop();
    void big_loop();
    void small_loop();
    void retire(cg::QueueReq *r, int status);
};

void cg_queue::retire(cg::QueueReq *r, int status) {
    // caller holds mu
    r->state = 2;
    r->status = status;
    r->res->status = status;
    in_use -= std::min(in_use, r->bytes);
    cv_done.notify_all();
}

void cg_queue::engine_loop() {
    hipStream_t stream = nullptr;
    std::unique_ptr<cg::BatchGroup> group;
    std::map<int, cg::QueueReq *> by_slot;
    try {
        CG_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
        const int cap = std::max(1, std::min(opts.max_active > 0 ? opts.max_active : 256, 4096));
        group.reset(new cg::BatchGroup(stream, cg::kSharedN, cap));
        std::vector<int> fin;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return stopping || !queued.empty() || !group->idle(); });
                if (stopping && group->idle()) break;
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
                        r->res->t_admit = r->res->t_done = cg::now_seconds();
                        r->res->t_submit = r->t_submit;
                        retire(r, CG_E_CANCELLED);
                        continue;
                    }
                    const int slot = group->free_slot();
                    if (slot < 0) break;
                    if (in_use + r->bytes > budget && !by_slot.empty()) break;
                    queued.pop_front();
                    in_use += r->bytes;
                    r->state = 1;
                    r->slot = slot;
                    group->add(slot, r->spec, r->res, r->t_submit, cg::now_seconds());
                    by_slot[slot] = r;
                }
            }
            if (!group->idle()) group->step(fin);
            std::lock_guard<std::mutex> lk(mu);
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
        for (auto *r : queued) retire(r, CG_E_DEVICE);
        queued.clear();
    }
    group.reset();
    if (stream) {
        (void)hipStreamSynchronize(stream);
        (void)hipStreamDestroy(stream);
    }
}

void cg_queue::big_loop() {
    std::unique_ptr<cg::Engine> eng;
    for (;;) {
        cg::QueueReq *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(mu);
            // admission: a large job starts when the budget allows it or no
            // other large job runs
            cv_work.wait(lk, [&] {
                return stopping || (!big_queued.empty() &&
                                    (big_running == 0 || in_use + big_queued.front()->bytes <= budget));
            });
            if (big_queued.empty()) break;
            r = big_queued.front();
            big_queued.pop_front();
            if (r->cancel || stopping) {
                r->res->t_submit = r->t_submit;
                r->res->t_admit = r->res->t_done = cg::now_seconds();
                r->bytes = 0;
                retire(r, CG_E_CANCELLED);
                continue;
            }
            r->state = 1;
            in_use += r->bytes;
            ++big_running;
        }
        const double t_admit = cg::now_seconds();
        int status;
        try {
            if (!eng) eng.reset(new cg::Engine(nullptr));
            eng->run(r->spec, r->res);
            status = r->res->status;
        } catch (const cg::Error &e) {
            status = e.code;
        } catch (...) {
            status = CG_E_DEVICE;
        }
        std::lock_guard<std::mutex> lk(mu);
        r->res->t_submit = r->t_submit;
        r->res->t_admit = t_admit;
        r->res->t_done = cg::now_seconds();
        --big_running;
        retire(r, status);
        cv_work.notify_all();  // budget freed: other large jobs may start
    }
}

// Small jobs (n <= 10, a permutation start): each launch of the small-job
// engine runs every such job queued at that moment, one workgroup per job;
// jobs that arrive meanwhile join the next launch. A job that has started
// runs to completion (a cancel then has no effect).
void cg_queue::small_loop() {
    hipStream_t stream = nullptr;
    std::unique_ptr<cg::WgRunner> runner;
    try {
        CG_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
        runner.reset(new cg::WgRunner(stream));
        for (;;) {
            std::vector<cg::QueueReq *> batch;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return stopping || !small_queued.empty(); });
                if (small_queued.empty()) break;
                while (!small_queued.empty()) {
                    cg::QueueReq *r = small_queued.front();
                    small_queued.pop_front();
                    if (r->cancel || stopping) {
                        r->res->t_submit = r->t_submit;
                        r->res->t_admit = r->res->t_done = cg::now_seconds();
                        retire(r, CG_E_CANCELLED);
                        continue;
                    }
                    r->state = 1;
                    in_use += r->bytes;
                    batch.push_back(r);
                }
            }
            if (batch.empty()) continue;
            std::vector<cg::WgItem> items;
            for (auto *r : batch) items.push_back({&r->spec, r->res});
            int status = CG_OK;
            try {
                cg::WgTuning t;
                runner->run(items, t, 0.0);
            } catch (const cg::Error &e) {
                status = e.code;
            }
            std::lock_guard<std::mutex> lk(mu);
            for (auto *r : batch) {
                r->res->t_submit = r->t_submit;
                retire(r, status == CG_OK ? r->res->status : status);
            }
        }
    } catch (const std::exception &e) {
        std::lock_guard<std::mutex> lk(mu);
        fatal = e.what();
        for (auto *r : small_queued) retire(r, CG_E_DEVICE);
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
        if (opts) q->opts = *opts;
        size_t free_b = 0, total_b = 0;
        CG_HIP(hipMemGetInfo(&free_b, &total_b));
        q->budget = q->opts.hbm_budget_bytes ? q->opts.hbm_budget_bytes : (uint64_t)(0.6 * (double)free_b);
        q->engine = std::thread([p = q.get()] { p->engine_loop(); });
        q->small_lane = std::thread([p = q.get()] { p->small_loop(); });
        const int lanes = q->opts.large_lanes > 0 ? std::min(q->opts.large_lanes, 8) : 2;
        for (int i = 0; i < lanes; ++i) q->big_lanes.emplace_back([p = q.get()] { p->big_loop(); });
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
    r->bytes = cg::estimate_bytes(r->spec);
    res_slot->status = CG_PENDING;
    std::lock_guard<std::mutex> lk(q->mu);
    if (!q->fatal.empty() || q->stopping) return CG_E_DEVICE;
    const int max_q = q->opts.max_queued > 0 ? q->opts.max_queued : 65536;
    if ((int)(q->queued.size() + q->big_queued.size() + q->small_queued.size()) >= max_q) return CG_E_BUSY;
    r->ticket = q->next_ticket++;
    // cheap jobs only: one workgroup runs the whole job, and a launch lasts
    // as long as its slowest job
    uint64_t states = 1;
    for (int i = 2; i <= r->spec.n; ++i) states *= (uint64_t)i;
    const bool small = r->spec.n <= cg::kWgMaxN && cg::wg_eligible(r->spec) &&
                       states * (uint64_t)std::max(1, r->spec.k) <= cg::kSmallLaneWork;
    if (small) r->bytes = 3 * ((states + 31) / 32) * 4;  // the job's three bitmaps
    // the shared group subtracts layers d and d-1 only: directed jobs that
    // are not small take a lane (its engine subtracts every visited state)
    r->big = !small && (!r->spec.inverse_closed || r->spec.n > cg::kSharedN ||
                        r->spec.orbit_bound > cg::kLargeOrbit || r->bytes > q->budget / 4);
    // large permutation jobs from n = 12 run in the bitmask engine: 3 bits
    // per state of S_n instead of 8-byte layers and candidate arrays (an
    // S_13 job holds 2.3 GB there); results are the same
    if (r->big && r->spec.n >= 12 && !(r->spec.flags & CG_PACKED_SORT) && cg::bitmask_unsupported(r->spec).empty()) {
        r->spec.flags |= CG_BITMASK;
        uint64_t states = 1;
        for (int i = 2; i <= r->spec.n; ++i) states *= (uint64_t)i;
        r->bytes = 3 * ((states + 31) / 32) * 4 + (64u << 20);
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
