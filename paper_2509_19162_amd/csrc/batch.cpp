// Batched growth (cg_growth_batch): independent jobs share super-steps.
//
// Workload shape: the paper's searches over many generating sets (section
// "Largest diameters found (and known) for n <= 15", exhaustive below n = 10
// and randomised above) run thousands of small, uneven growth jobs. One
// super-step advances every running job of a group by one layer with a
// single expand, sort, unique + set difference and compaction over
// job-tagged keys; a job's result equals its stand-alone result because
// tags keep the jobs' states apart.
#include "batch.h"

#include <cstdio>
#include <cstdlib>
#include <mutex>

#include "bitmap.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <string>

namespace cg {

BatchGroup::BatchGroup(hipStream_t stream, int n_max, int slots) : stream_(stream), n_max_(n_max) {
    if (slots < 1) slots = 1;
    tag_bits_ = 0;
    while ((1 << tag_bits_) < slots) ++tag_bits_;
    shift_ = 4 * n_max;
    if (shift_ + tag_bits_ > 64) throw Error(CG_E_INVAL, "too many jobs for the key width of this n");
    slot_.resize(slots);
    quarantine_.assign(slots, 0);
    w_.init(stream_);
    for (DevBuf *b : {&gsel_, &jobs_, &cand0_, &cand1_, &lay_[0], &lay_[1], &lay_[2], &cnt_, &pos_, &join_,
                      &merged_})
        b->stream = stream_;
    host_cap_ = (size_t)slots + 8;
    CG_HIP(hipHostMalloc((void **)&host_, host_cap_ * sizeof(uint64_t), hipHostMallocDefault));
    cnt_.ensure((size_t)slots * sizeof(uint64_t));
    pos_.ensure(((size_t)slots + 1) * sizeof(uint64_t));
    jobs_.ensure((size_t)slots * sizeof(BatchJobDev));
    for (int i = 0; i < 3; ++i) lay_[i].ensure(1024);
}

BatchGroup::~BatchGroup() {
    (void)hipStreamSynchronize(stream_);
    if (host_) (void)hipHostFree(host_);
}

int BatchGroup::free_slot() const {
    for (int s = 0; s < (int)slot_.size(); ++s)
        if (!slot_[s].res && quarantine_[s] == 0) return s;
    return -1;
}

bool BatchGroup::idle() const {
    for (auto &j : slot_)
        if (j.res) return false;
    return pending_keys_.empty();
}

uint64_t BatchGroup::device_bytes() const {
    uint64_t b = cand0_.bytes + cand1_.bytes + merged_.bytes + join_.bytes + gsel_.bytes + jobs_.bytes + cnt_.bytes +
                 pos_.bytes;
    for (const DevBuf *x : {&w_.hist, &w_.base, &w_.small, &w_.status, &w_.bounds, &w_.tile_cnt, &w_.tile_off,
                            &w_.kill, &w_.tcnt, &w_.toff, &w_.bsum})
        b += x->bytes;
    for (int i = 0; i < 3; ++i) b += lay_[i].bytes;
    return b;
}

bool BatchGroup::release_idle() {
    if (!idle()) return false;
    CG_HIP(hipStreamSynchronize(stream_));
    for (DevBuf *x : {&cand0_, &cand1_, &merged_, &join_, &w_.status, &w_.bounds, &w_.tile_cnt, &w_.tile_off,
                      &w_.kill, &w_.tcnt, &w_.toff, &w_.bsum})
        x->release();
    w_.epoch = 0;
    for (int i = 0; i < 3; ++i) {
        lay_[i].release();
        lay_[i].ensure(1024);
    }
    ncur_ = nprev_ = 0;
    std::fill(quarantine_.begin(), quarantine_.end(), 0);  // no key of a finished job is left
    for (auto &J : slot_) J.F = 0;
    return true;
}

void BatchGroup::add(int slot, const JobSpec &spec, cg_result_t *res, double t_submit, double t_admit) {
    if (slot < 0 || slot >= (int)slot_.size() || slot_[slot].res || quarantine_[slot])
        throw Error(CG_E_INVAL, "slot not free");
    if (spec.n > n_max_) throw Error(CG_E_INVAL, "job n exceeds the group's n");
    SlotJob &J = slot_[slot];
    J = SlotJob{};
    J.spec = spec;
    J.res = res;
    J.t_submit = t_submit;
    J.t_admit = t_admit;
    J.F = 0;  // its start key joins the frontier at the next step
    J.layers = 1;
    std::memset(res->layer_sizes, 0, sizeof(uint64_t) * (size_t)spec.max_layers);
    res->layer_sizes[0] = 1;
    res->states_expanded = 0;
    res->candidates = 0;
    res->n_kstats = 0;
    res->device_ms = 0;
    const uint64_t tag = shift_ >= 64 ? 0 : ((uint64_t)slot << shift_);
    J.key0 = tag | pack_host(spec.n, spec.start);
    pending_keys_.push_back(J.key0);
    sel_dirty_ = true;
}

void BatchGroup::finish(int slot, int status) {
    SlotJob &J = slot_[slot];
    cg_result_t *r = J.res;
    r->status = status;
    r->num_layers = J.layers;
    r->t_submit = J.t_submit;
    r->t_admit = J.t_admit;
    r->t_done = now_seconds();
    J.res = nullptr;
    J.done = true;
    quarantine_[slot] = 3;  // its keys may still sit in layers d and d-1
}

void BatchGroup::cancel(int slot) {
    if (!occupied(slot)) return;
    SlotJob &J = slot_[slot];
    if (J.F == 0 && J.layers == 1) {
        // not merged into the frontier yet: withdraw the start key
        auto it = std::find(pending_keys_.begin(), pending_keys_.end(), J.key0);
        if (it != pending_keys_.end()) pending_keys_.erase(it);
    }
    finish(slot, CG_E_CANCELLED);
}

void BatchGroup::rebuild_gensel() {
    hsel_.clear();
    for (auto &J : slot_) {
        J.goff = (uint32_t)hsel_.size();
        if (!J.res) continue;
        for (int g = 0; g < J.spec.k; ++g) hsel_.push_back(make_gensel(J.spec.n, J.spec.gens.data() + (size_t)g * J.spec.n));
    }
    if (hsel_.empty()) hsel_.push_back(GenSel{});
    gsel_.ensure(sizeof(GenSel) * hsel_.size(), 1.5);
    CG_HIP(hipMemcpyAsync(gsel_.p, hsel_.data(), sizeof(GenSel) * hsel_.size(), hipMemcpyHostToDevice, stream_));
    sel_dirty_ = false;
}

void BatchGroup::step(std::vector<int> &finished) {
    finished.clear();
    // 1. joining jobs: their start keys merge into the current layer
    if (!pending_keys_.empty()) {
        std::sort(pending_keys_.begin(), pending_keys_.end());
        const uint64_t np = pending_keys_.size();
        join_.fit(np * sizeof(uint64_t), 1.5);
        CG_HIP(hipMemcpyAsync(join_.p, pending_keys_.data(), np * sizeof(uint64_t), hipMemcpyHostToDevice,
                              stream_));
        merged_.fit((ncur_ + np) * sizeof(uint64_t), 1.5);
        launch_merge(lay_[ic_].as<uint64_t>(), ncur_, join_.as<uint64_t>(), np, merged_.as<uint64_t>(), stream_);
        lay_[ic_].swap(merged_);
        ncur_ += np;
        for (auto &J : slot_)
            if (J.res && J.F == 0 && J.layers == 1 && !J.done) J.F = 1;
        CG_HIP(hipStreamSynchronize(stream_));  // pending_keys_ is host memory
        pending_keys_.clear();
    }
    if (sel_dirty_) rebuild_gensel();

    // 2. stop rules, job table
    const int S = (int)slot_.size();
    std::vector<BatchJobDev> tab(S);
    uint64_t foff = 0, coff = 0;
    bool any = false;
    for (int s = 0; s < S; ++s) {
        SlotJob &J = slot_[s];
        BatchJobDev &d = tab[s];
        d.front_off = foff;
        d.cand_off = coff;
        d.goff = J.goff;
        d.kk = 0;
        if (J.res) {
            const bool stop = J.layers >= J.spec.max_layers ||
                              (J.spec.max_frontier && J.F > J.spec.max_frontier) || J.spec.k == 0;
            if (stop) {
                finish(s, J.spec.k == 0 ? CG_OK : CG_TRUNCATED);
                finished.push_back(s);
            } else {
                d.kk = (uint32_t)J.spec.k;
                any = true;
            }
        }
        foff += J.F;
        coff += (uint64_t)d.kk * J.F;
    }
    if (foff != ncur_) throw Error(CG_E_DEVICE, "batch bookkeeping: frontier size mismatch");
    const uint64_t C = coff;
    if (!any) {
        // nothing expands: the layers rotate empty so lingering keys age out
        for (auto &J : slot_) J.F = 0;
        std::swap(ip_, ic_);
        nprev_ = ncur_;
        ncur_ = 0;
        for (int s = 0; s < S; ++s)
            if (quarantine_[s]) --quarantine_[s];
        return;
    }
    CG_HIP(hipMemcpyAsync(jobs_.p, tab.data(), sizeof(BatchJobDev) * S, hipMemcpyHostToDevice, stream_));

    // 3. expand, sort, unique + set difference, compaction, per-job counts
    cand0_.fit(C * sizeof(uint64_t) + 64, 1.25);
    cand1_.fit(C * sizeof(uint64_t) + 64, 1.25);
    launch_batch_expand(lay_[ic_].as<uint64_t>(), ncur_, jobs_.as<BatchJobDev>(), gsel_.as<GenSel>(),
                        cand0_.as<uint64_t>(), shift_, C, (uint32_t)S, w_);
    const int hi = std::min(64, shift_ + tag_bits_);
    uint64_t *sorted = radix_sort(cand0_.as<uint64_t>(), cand1_.as<uint64_t>(), C, 4, hi, w_);
    uint64_t *scratch = sorted == cand0_.as<uint64_t>() ? cand1_.as<uint64_t>() : cand0_.as<uint64_t>();
    launch_dedup_count(sorted, C, lay_[ic_].as<uint64_t>(), ncur_, lay_[ip_].as<uint64_t>(), nprev_, scratch,
                       w_.counter(), w_);
    // the new layer is sized once its length is known
    CG_HIP(hipMemcpyAsync(host_, w_.counter(), sizeof(uint64_t), hipMemcpyDeviceToHost, stream_));
    CG_HIP(hipMemcpyAsync(host_ + 1, w_.err(), sizeof(uint32_t), hipMemcpyDeviceToHost, stream_));
    CG_HIP(hipStreamSynchronize(stream_));
    const uint64_t N = host_[0];
    if (((uint32_t *)(host_ + 1))[0] != 0) throw Error(CG_E_DEVICE, "kernel error flag set in a batch step");
    if (N > C) throw Error(CG_E_DEVICE, "batch layer size out of range");
    lay_[in_].fit(std::max<uint64_t>(N, 1) * sizeof(uint64_t) + 64, 1.25);
    launch_dedup_gather(scratch, lay_[in_].as<uint64_t>(), N, w_);
    launch_tag_count(lay_[in_].as<uint64_t>(), N, shift_, cnt_.as<unsigned long long>(),
                     pos_.as<unsigned long long>(), (uint32_t)S, w_);
    CG_HIP(hipMemcpyAsync(host_ + 2, cnt_.p, sizeof(uint64_t) * S, hipMemcpyDeviceToHost, stream_));
    CG_HIP(hipMemcpyAsync(host_ + 1, w_.err(), sizeof(uint32_t), hipMemcpyDeviceToHost, stream_));
    CG_HIP(hipStreamSynchronize(stream_));
    if (((uint32_t *)(host_ + 1))[0] != 0) throw Error(CG_E_DEVICE, "kernel error flag set in a batch step");

    // 4. per-job bookkeeping
    uint64_t sum = 0;
    for (int s = 0; s < S; ++s) {
        SlotJob &J = slot_[s];
        const uint64_t Ns = host_[2 + s];
        sum += Ns;
        if (tab[s].kk == 0) {
            if (Ns) throw Error(CG_E_DEVICE, "a job that did not expand produced states");
            J.F = 0;
            continue;
        }
        J.res->states_expanded += J.F;
        J.res->candidates += (uint64_t)tab[s].kk * J.F;
        J.F = Ns;
        if (Ns == 0) {
            finish(s, CG_OK);
            finished.push_back(s);
        } else {
            J.res->layer_sizes[J.layers++] = Ns;
        }
    }
    if (sum != N) throw Error(CG_E_DEVICE, "per-job counts do not add up to the layer size");
    // 5. rotate layers
    const int t = ip_;
    ip_ = ic_;
    ic_ = in_;
    in_ = t;
    nprev_ = ncur_;
    ncur_ = N;
    for (int s = 0; s < S; ++s)
        if (quarantine_[s] && !slot_[s].res) --quarantine_[s];
}

}  // namespace cg

namespace cg {

// Size classes of a batch are the job's n. Per class the batch picks an
// engine: the small-job engine (one workgroup per job, every such job of
// the batch in one persistent launch, built as a hipGraph that replays while
// the batch's shape repeats) or tagged super-step groups of at most `cap`
// jobs. A job far above its share of the small-job work leaves that engine
// for a group (one workgroup would run it long after the rest finished).
// Defaults: small-job engine up to n = wg_max_n (CG_WG_MAX_N, default 10),
// workgroup size by n, groups of up to 4096 jobs, the heavy-job split at
// 1/64 of the small-job work. With opts->tune the autotuner times the
// choices on the batch itself: per class, both engines, three workgroup
// sizes and two group sizes on a sample of up to 256 jobs; for the whole
// batch, three heavy-job splits. Its choices are kept per device model in
// a file (CG_TUNE_CACHE, default $XDG_CACHE_HOME or ~/.cache, then
// cayleygrowth_tune.txt) and reused by later batches and processes.
// Results are exact whatever is chosen.
namespace {

int default_wg_max_n() {
    const char *e = std::getenv("CG_WG_MAX_N");
    if (!e) return kWgMaxN;
    return std::max(0, std::min(kWgMaxN, std::atoi(e)));
}

struct ClassChoice {
    bool wg = true;        // small-job engine (else tagged groups)
    int block = 256;       // its workgroup size
    int group_cap = 4096;  // jobs per tagged group
};

// What a cg_growth_batch call keeps on a device between calls: a stream,
// the small-job runner (so its launch graph replays while the shape
// repeats) and the autotuner's choices.
struct BatchContext {
    std::mutex mu;
    int dev = 0;
    hipStream_t stream = nullptr;
    std::unique_ptr<WgRunner> runner;
    std::string model;                 // device model the choices belong to
    std::map<int, ClassChoice> tuned;  // by n
    double heavy_div = 0;              // 0: not tuned
    bool loaded = false;
    uint64_t calls = 0;
    int file_entries = 0;
};

struct BatchContexts {
    std::mutex mu;
    std::map<int, BatchContext *> ctx;  // never destroyed: their streams live until exit
};

BatchContexts &batch_contexts() {
    static BatchContexts c;
    return c;
}

BatchContext &batch_context(int dev) {
    BatchContexts &all = batch_contexts();
    std::lock_guard<std::mutex> lk(all.mu);
    BatchContext *&c = all.ctx[dev];
    if (!c) {
        c = new BatchContext();
        c->dev = dev;
        hipDeviceProp_t prop{};
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess)
            c->model = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) + "cu";
        else
            c->model = "unknown";
        for (char &ch : c->model)
            if (ch == ' ' || ch == '\n') ch = '_';
    }
    return *c;
}

std::string tune_cache_path() {
    if (const char *e = std::getenv("CG_TUNE_CACHE")) return e;
    std::string dir;
    if (const char *x = std::getenv("XDG_CACHE_HOME"))
        dir = x;
    else if (const char *h = std::getenv("HOME"))
        dir = std::string(h) + "/.cache";
    else
        return "";
    return dir + "/cayleygrowth_tune.txt";
}

// File format, one choice per line: "<model> class <n> <wg> <block> <cap>"
// or "<model> heavy <divisor>"; the last line for a key wins.
void load_tuning(BatchContext &c) {
    c.loaded = true;
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return;
    char model[128], kind[16];
    while (std::fscanf(f, "%127s %15s", model, kind) == 2) {
        if (c.model != model) {
            int ch;
            while ((ch = std::fgetc(f)) != EOF && ch != '\n') {
            }
            continue;
        }
        if (std::strcmp(kind, "class") == 0) {
            int n, wg, block, cap;
            if (std::fscanf(f, "%d %d %d %d", &n, &wg, &block, &cap) != 4) break;
            if (n < 1 || n > 16 || block < 64 || block > 1024 || block % 64 || cap < 1) continue;
            c.tuned[n] = ClassChoice{wg != 0, block, cap};
            ++c.file_entries;
        } else if (std::strcmp(kind, "heavy") == 0) {
            double d;
            if (std::fscanf(f, "%lf", &d) != 1) break;
            if (d >= 1) {
                c.heavy_div = d;
                ++c.file_entries;
            }
        }
    }
    std::fclose(f);
}

void save_tuning(const BatchContext &c) {
    const std::string path = tune_cache_path();
    if (path.empty()) return;
    FILE *f = std::fopen(path.c_str(), "a");
    if (!f) return;  // an unwritable cache only costs a re-tune
    for (auto &kv : c.tuned)
        std::fprintf(f, "%s class %d %d %d %d\n", c.model.c_str(), kv.first, kv.second.wg ? 1 : 0, kv.second.block,
                     kv.second.group_cap);
    if (c.heavy_div > 0) std::fprintf(f, "%s heavy %g\n", c.model.c_str(), c.heavy_div);
    std::fclose(f);
}

double time_groups(std::vector<std::pair<JobSpec, cg_result_t *>> &sample, int n, int cap, hipStream_t stream) {
    const double t = now_seconds();
    for (size_t base = 0; base < sample.size(); base += (size_t)cap) {
        const int m = (int)std::min<size_t>((size_t)cap, sample.size() - base);
        BatchGroup g(stream, n, m);
        for (int j = 0; j < m; ++j) g.add(j, sample[base + j].first, sample[base + j].second, t, t);
        std::vector<int> fin;
        while (!g.idle()) g.step(fin);
    }
    CG_HIP(hipStreamSynchronize(stream));
    return now_seconds() - t;
}

int group_cap_for(int n) {
    int cap = 1;
    while (4 * n + 1 + (int)std::log2((double)cap) <= 64 && cap < 4096) cap <<= 1;
    if (4 * n >= 64) cap = 1;
    return cap;
}

// Times the choices for one class on up to 256 of its jobs.
ClassChoice tune_class(int n, std::vector<std::pair<JobSpec, cg_result_t *>> &items, BatchContext &c) {
    const size_t m = std::min<size_t>(256, items.size());
    std::vector<std::pair<JobSpec, cg_result_t *>> sample;
    std::vector<std::vector<uint64_t>> sizes(m);
    std::vector<cg_result_t> res(m);
    for (size_t i = 0; i < m; ++i) {
        sizes[i].assign((size_t)items[i].first.max_layers, 0);
        std::memset(&res[i], 0, sizeof(cg_result_t));
        res[i].layer_sizes = sizes[i].data();
        sample.push_back({items[i].first, &res[i]});
    }
    std::vector<WgItem> wi;
    for (auto &x : sample) wi.push_back({&x.first, x.second});
    ClassChoice ch;
    double t0 = now_seconds();
    double dev_ms = 0;
    ch.block = tune_wg(wi, *c.runner, &dev_ms).block;
    WgTuning t;
    t.block = ch.block;
    t0 = now_seconds();
    c.runner->run(wi, t, t0);
    const double wg_s = now_seconds() - t0;
    double grp_s = -1;
    const int cap_max = group_cap_for(n);
    for (int cap : {std::min(512, cap_max), cap_max}) {
        (void)time_groups(sample, n, cap, c.stream);  // warm-up (allocations)
        const double g = time_groups(sample, n, cap, c.stream);
        if (grp_s < 0 || g < grp_s) {
            grp_s = g;
            ch.group_cap = cap;
        }
    }
    ch.wg = wg_s <= grp_s;
    if (std::getenv("CG_TUNE_LOG"))
        std::fprintf(stderr, "[tune] n=%d sample=%zu workgroup=%d wg %.2f ms, groups(cap %d) %.2f ms -> %s\n", n, m,
                     ch.block, 1e3 * wg_s, ch.group_cap, 1e3 * grp_s, ch.wg ? "workgroups" : "groups");
    return ch;
}

struct Item {
    int idx;
    JobSpec spec;
};

uint64_t job_work(const JobSpec &sp) {
    uint64_t w = (uint64_t)std::max(1, sp.k);
    for (int i = 2; i <= sp.n; ++i) w *= (uint64_t)i;
    return w;
}

// One batch with the given choices (classes without a tuned entry take the
// defaults). Returns the seconds it took.
double run_with(std::map<int, std::vector<Item>> &by_n, cg_result_t *results, const cg_batch_opts_t *opts,
                BatchContext &c, bool use_tuned, double heavy_div, double t0) {
    const double ts = now_seconds();
    hipStream_t stream = c.stream;
    const int wg_max_n = default_wg_max_n();
    double wg_total = 0;
    for (auto &kv : by_n)
        for (auto &it : kv.second)
            if (wg_eligible(it.spec)) wg_total += (double)job_work(it.spec);
    const double heavy = std::max((double)(1ull << 22), wg_total / heavy_div);
    std::vector<WgItem> wg_items;
    std::vector<Item *> alone;
    WgTuning wg_t;
    int wg_t_n = -1;
    for (auto &kv : by_n) {
        const int n = kv.first;
        auto &all = kv.second;
        ClassChoice ch;
        ch.wg = n <= wg_max_n;
        ch.block = n >= 10 ? 1024 : (n == 9 ? 512 : 256);  // the autotuner's usual picks on MI355X
        ch.group_cap = group_cap_for(n);
        if (use_tuned) {
            auto f = c.tuned.find(n);
            if (f != c.tuned.end()) ch = f->second;
        }
        std::vector<Item> items;
        for (auto &it : all) {
            const bool heavy_job = (double)job_work(it.spec) > heavy;
            if (wg_eligible(it.spec) && (!it.spec.inverse_closed || (ch.wg && !heavy_job))) {
                wg_items.push_back({&it.spec, &results[it.idx]});
                if (n > wg_t_n) {
                    wg_t_n = n;
                    wg_t.block = ch.block;
                }
            } else if (!it.spec.inverse_closed) {
                alone.push_back(&it);  // groups subtract two layers only
            } else {
                items.push_back(it);
            }
        }
        if (items.empty()) continue;
        int cap = std::min(ch.group_cap, group_cap_for(n));
        if (opts && opts->max_active > 0) cap = std::min(cap, opts->max_active);
        // groups of at most `cap` jobs; a group that runs out of device
        // memory is split in half and its jobs start over
        std::vector<std::pair<size_t, size_t>> todo;
        for (size_t base = 0; base < items.size(); base += (size_t)cap)
            todo.push_back({base, std::min<size_t>((size_t)cap, items.size() - base)});
        while (!todo.empty()) {
            const auto span = todo.back();
            todo.pop_back();
            const int m = (int)span.second;
            try {
                BatchGroup g(stream, n, m);
                for (int j = 0; j < m; ++j) {
                    Item &it = items[span.first + j];
                    g.add(j, it.spec, &results[it.idx], t0, now_seconds());
                }
                std::vector<int> fin;
                while (!g.idle()) g.step(fin);
            } catch (const Error &e) {
                if (e.code != CG_E_NOMEM || m == 1) throw;
                CG_HIP(hipStreamSynchronize(stream));
                todo.push_back({span.first + (size_t)m / 2, (size_t)(m - m / 2)});
                todo.push_back({span.first, (size_t)m / 2});
            }
        }
    }
    if (!alone.empty()) {
        // directed jobs the small-job engine cannot take: one engine, one
        // job after the other (every visited state subtracted)
        Engine eng(stream);
        for (Item *it : alone) {
            cg_result_t *r = &results[it->idx];
            try {
                eng.run(it->spec, r);
            } catch (const Error &e) {
                r->status = e.code;
                r->num_layers = 0;
            }
        }
    }
    if (const char *e = std::getenv("CG_WG_BLOCK")) wg_t.block = std::atoi(e);
    if (!wg_items.empty()) c.runner->run(wg_items, wg_t, t0);  // one persistent launch for every small job
    CG_HIP(hipStreamSynchronize(stream));
    return now_seconds() - ts;
}

}  // namespace

void run_batch(int n_jobs, const cg_job_t *jobs, cg_result_t *results, const cg_batch_opts_t *opts) {
    const double t0 = now_seconds();
    int dev = 0;
    CG_HIP(hipGetDevice(&dev));
    BatchContext &c = batch_context(dev);
    std::lock_guard<std::mutex> lk(c.mu);  // one batch at a time per device
    if (!c.stream) CG_HIP(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
    if (!c.runner) c.runner.reset(new WgRunner(c.stream));
    ++c.calls;
    // work already queued on the caller's stream comes first
    hipStream_t user = opts ? (hipStream_t)opts->stream : nullptr;
    if (user) {
        hipEvent_t e;
        CG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        CG_HIP(hipEventRecord(e, user));
        CG_HIP(hipStreamWaitEvent(c.stream, e, 0));
        (void)hipEventDestroy(e);
    }
    std::map<int, std::vector<Item>> by_n;
    for (int i = 0; i < n_jobs; ++i) {
        cg_result_t *r = &results[i];
        if (!r->layer_sizes) {
            r->status = CG_E_INVAL;
            continue;
        }
        try {
            JobSpec s = canonicalize(jobs[i], true);
            by_n[s.n].push_back({i, std::move(s)});
        } catch (const Error &e) {
            r->status = e.code;
            r->num_layers = 0;
        }
    }
    const bool tune = opts && opts->tune;
    if (!tune) {
        (void)run_with(by_n, results, opts, c, false, 64.0, t0);
        return;
    }
    if (!c.loaded) load_tuning(c);
    bool changed = false;
    for (auto &kv : by_n) {
        const int n = kv.first;
        if (c.tuned.count(n)) continue;
        std::vector<std::pair<JobSpec, cg_result_t *>> cls;
        bool wg_all = true;
        for (auto &it : kv.second) {
            if (!wg_eligible(it.spec) || !it.spec.inverse_closed) wg_all = false;
            cls.push_back({it.spec, &results[it.idx]});
        }
        if (!wg_all || n > default_wg_max_n()) continue;  // the defaults are the only choice
        c.tuned[n] = tune_class(n, cls, c);
        changed = true;
    }
    if (c.heavy_div <= 0) {
        // the heavy-job split: each candidate on the whole batch
        double best = -1;
        for (double d : {16.0, 64.0, 256.0}) {
            const double s = run_with(by_n, results, opts, c, true, d, t0);
            if (std::getenv("CG_TUNE_LOG")) std::fprintf(stderr, "[tune] heavy split 1/%g: %.2f ms\n", d, 1e3 * s);
            if (best < 0 || s < best) {
                best = s;
                c.heavy_div = d;
            }
        }
        changed = true;
    }
    if (changed) save_tuning(c);
    (void)run_with(by_n, results, opts, c, true, c.heavy_div, t0);
}

void release_batch_buffers() {
    BatchContexts &all = batch_contexts();
    std::lock_guard<std::mutex> lk(all.mu);
    for (auto &kv : all.ctx) {
        BatchContext &c = *kv.second;
        std::lock_guard<std::mutex> l2(c.mu);  // waits for a batch call in progress
        if (c.runner) c.runner->release();
    }
}

void batch_info(cg_batch_info_t *out) {
    int dev = 0;
    CG_HIP(hipGetDevice(&dev));
    BatchContext &c = batch_context(dev);
    std::lock_guard<std::mutex> lk(c.mu);
    std::memset(out, 0, sizeof *out);
    out->calls = c.calls;
    if (c.runner) {
        out->graph_builds = (uint64_t)c.runner->graph_captures();
        out->graph_launches = (uint64_t)c.runner->graph_launches();
    }
    out->tuned_classes = (int)c.tuned.size();
    out->heavy_split = c.heavy_div;
    out->tune_file_entries = c.file_entries;
}

}  // namespace cg
