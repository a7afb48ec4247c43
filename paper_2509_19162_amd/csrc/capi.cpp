// The C ABI of libcayleygrowth.so (include/cayleygrowth.h and
// include/cayleygrowth_testing.h). Every entry point catches everything:
// no C++ exception crosses the boundary; failures become CG_E_* codes with
// a thread-local detail string.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/cayleygrowth.h"
#include "../../include/cayleygrowth_testing.h"
#include "batch.h"
#include "bitmap.h"
#include "engine.h"
#include "perm_rank.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

template <class F>
int guarded(F &&f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const cg::Error &e) {
        return fail(e.code, e.what());
    } catch (const std::bad_alloc &) {
        return fail(CG_E_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(CG_E_DEVICE, e.what());
    } catch (...) {
        return fail(CG_E_DEVICE, "unknown failure");
    }
}

}  // namespace

namespace cg {
void set_last_error(const std::string &msg) { g_last_error = msg; }
}  // namespace cg

extern "C" {

const char *cg_strerror(int code) {
    switch (code) {
        case CG_OK: return "complete";
        case CG_TRUNCATED: return "truncated by a stop rule";
        case CG_PENDING: return "pending";
        case CG_E_INVAL: return "invalid argument";
        case CG_E_NOMEM: return "out of memory";
        case CG_E_DEVICE: return "device error";
        case CG_E_UNSUPPORTED: return "unsupported generating set";
        case CG_E_BUSY: return "busy (queue full, or buffers still in use)";
        case CG_E_CANCELLED: return "cancelled";
        case CG_E_TIMEOUT: return "timed out";
        default: return "unknown status";
    }
}

const char *cg_last_error(void) { return g_last_error.c_str(); }

void cg_release_cached_memory(void) {
    guarded([&]() -> int {
        cg::release_batch_buffers();
        cg::release_cached_device_memory();
        return CG_OK;
    });
}

int cg_growth_ex(const cg_job_t *job, cg_result_t *res, void *stream) {
    return guarded([&]() -> int {
        if (!job || !res || !res->layer_sizes) throw cg::Error(CG_E_INVAL, "NULL job or result");
        const cg::JobSpec spec = cg::canonicalize(*job, false);
        cg::Engine eng((hipStream_t)stream);
        eng.run(spec, res);
        return res->status;
    });
}

int cg_growth(int n, const uint8_t *gens, int n_gens, int max_layers, uint64_t *out_layer_sizes) {
    if (!out_layer_sizes) return fail(CG_E_INVAL, "NULL out_layer_sizes");
    cg_job_t job{};
    job.n = n;
    job.gens = gens;
    job.n_gens = n_gens;
    job.max_layers = max_layers;
    cg_result_t res{};
    res.layer_sizes = out_layer_sizes;
    return cg_growth_ex(&job, &res, nullptr);
}

int cg_memory_stats(cg_memory_stats_t *out, int reset_peak) {
    return guarded([&]() -> int {
        if (!out) throw cg::Error(CG_E_INVAL, "NULL result");
        cg::memory_stats(out, reset_peak != 0);
        return CG_OK;
    });
}

int cg_set_workspace(void *dev_ptr, size_t bytes) {
    return guarded([&]() -> int {
        cg::release_batch_buffers();  // the batches' kept buffers may live in the old arena
        cg::set_workspace(dev_ptr, bytes);
        return CG_OK;
    });
}

int cg_growth_stats(const uint64_t *sizes, int num_layers, cg_growth_stats_t *out) {
    return guarded([&]() -> int {
        if (!sizes || !out || num_layers < 1) throw cg::Error(CG_E_INVAL, "NULL sizes or result, or no layers");
        cg::growth_stats(sizes, num_layers, out);
        return CG_OK;
    });
}

int cg_growth_batch(int n_jobs, const cg_job_t *jobs, cg_result_t *results, const cg_batch_opts_t *opts) {
    return guarded([&]() -> int {
        if (n_jobs < 0 || (n_jobs > 0 && (!jobs || !results)))
            throw cg::Error(CG_E_INVAL, "bad batch arguments");
        cg::run_batch(n_jobs, jobs, results, opts);
        return CG_OK;
    });
}

int cg_batch_info(cg_batch_info_t *out) {
    return guarded([&]() -> int {
        if (!out) throw cg::Error(CG_E_INVAL, "NULL batch info");
        cg::batch_info(out);
        return CG_OK;
    });
}

int cg_growth_batch_noalloc(int n_jobs, const cg_job_t *jobs, cg_result_t *results, void *stream) {
    return guarded([&]() -> int {
        if (n_jobs < 0 || (n_jobs > 0 && (!jobs || !results)))
            throw cg::Error(CG_E_INVAL, "bad batch arguments");
        cg::run_batch_noalloc(n_jobs, jobs, results, (hipStream_t)stream);
        return CG_OK;
    });
}

struct cg_engine {
    cg::Engine eng;
    explicit cg_engine(hipStream_t s) : eng(s) {}
};

cg_engine_t *cg_engine_create(void *stream) {
    cg_engine_t *e = nullptr;
    const int rc = guarded([&]() -> int {
        e = new cg_engine((hipStream_t)stream);
        return CG_OK;
    });
    return rc == CG_OK ? e : nullptr;
}

int cg_engine_run(cg_engine_t *e, const cg_job_t *job, cg_result_t *res) {
    return guarded([&]() -> int {
        if (!e || !job || !res || !res->layer_sizes) throw cg::Error(CG_E_INVAL, "NULL engine, job or result");
        const cg::JobSpec spec = cg::canonicalize(*job, false);
        e->eng.run(spec, res);
        return res->status;
    });
}

void cg_engine_destroy(cg_engine_t *e) {
    guarded([&]() -> int {
        delete e;
        return CG_OK;
    });
}

// ---- kernel-level test entry points -------------------------------------------

int cg_test_pack(int n, const uint8_t *h_states, uint64_t count, uint64_t *d_keys, void *stream) {
    return guarded([&]() -> int {
        if (n < 1 || n > 16 || (!h_states && count) || (!d_keys && count))
            throw cg::Error(CG_E_INVAL, "bad pack arguments");
        if (!count) return CG_OK;
        hipStream_t s = (hipStream_t)stream;
        cg::DevBuf rows;
        rows.stream = s;
        rows.ensure(count * n);
        CG_HIP(hipMemcpyAsync(rows.p, h_states, count * n, hipMemcpyHostToDevice, s));
        cg::launch_pack(n, rows.as<uint8_t>(), count, d_keys, s);
        CG_HIP(hipStreamSynchronize(s));
        return CG_OK;
    });
}

int cg_test_unpack(int n, const uint64_t *d_keys, uint64_t count, uint8_t *h_states, void *stream) {
    return guarded([&]() -> int {
        if (n < 1 || n > 16 || (!h_states && count) || (!d_keys && count))
            throw cg::Error(CG_E_INVAL, "bad unpack arguments");
        if (!count) return CG_OK;
        hipStream_t s = (hipStream_t)stream;
        cg::DevBuf rows;
        rows.stream = s;
        rows.ensure(count * n);
        cg::launch_unpack(n, d_keys, count, rows.as<uint8_t>(), s);
        CG_HIP(hipMemcpyAsync(h_states, rows.p, count * n, hipMemcpyDeviceToHost, s));
        CG_HIP(hipStreamSynchronize(s));
        return CG_OK;
    });
}

static std::vector<cg::GenSel> make_sels(int n, const uint8_t *h_gens, int k) {
    if (n < 1 || n > 16 || k < 1 || !h_gens) throw cg::Error(CG_E_INVAL, "bad generator arguments");
    std::vector<cg::GenSel> v(k);
    for (int g = 0; g < k; ++g) {
        bool seen[16] = {false};
        for (int i = 0; i < n; ++i) {
            const uint8_t x = h_gens[(size_t)g * n + i];
            if (x >= n || seen[x]) throw cg::Error(CG_E_INVAL, "generator row is not a permutation");
            seen[x] = true;
        }
        v[g] = cg::make_gensel(n, h_gens + (size_t)g * n);
    }
    return v;
}

int cg_test_expand(int n, const uint8_t *h_gens, int k, const uint64_t *d_frontier, uint64_t F,
                   uint64_t *d_out, void *stream) {
    return guarded([&]() -> int {
        auto sels = make_sels(n, h_gens, k);
        if (F && (!d_frontier || !d_out)) throw cg::Error(CG_E_INVAL, "NULL device pointer");
        hipStream_t s = (hipStream_t)stream;
        cg::PipeWork w;
        w.init(s);
        cg::DevBuf gs;
        gs.stream = s;
        gs.ensure(sizeof(cg::GenSel) * k);
        CG_HIP(hipMemcpyAsync(gs.p, sels.data(), sizeof(cg::GenSel) * k, hipMemcpyHostToDevice, s));
        cg::launch_expand(d_frontier, F, gs.as<cg::GenSel>(), k, d_out, w);
        CG_HIP(hipStreamSynchronize(s));
        return CG_OK;
    });
}

int cg_test_sort(uint64_t *d_keys, uint64_t *d_tmp, uint64_t count, int bit_lo, int bit_hi,
                 void *stream) {
    return guarded([&]() -> int {
        if (bit_lo < 0 || bit_hi > 64 || bit_lo >= bit_hi) throw cg::Error(CG_E_INVAL, "bad bit range");
        if (cg::sort_passes(bit_lo, bit_hi) > cg::kMaxPasses)
            throw cg::Error(CG_E_INVAL, "bit range needs more than 8 passes");
        if (count && (!d_keys || !d_tmp)) throw cg::Error(CG_E_INVAL, "NULL device pointer");
        hipStream_t s = (hipStream_t)stream;
        cg::PipeWork w;
        w.init(s);
        uint64_t *res = cg::radix_sort(d_keys, d_tmp, count, bit_lo, bit_hi, w);
        if (res != d_keys)
            CG_HIP(hipMemcpyAsync(d_keys, res, count * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        uint32_t err = 0;
        CG_HIP(hipMemcpyAsync(&err, w.err(), sizeof err, hipMemcpyDeviceToHost, s));
        CG_HIP(hipStreamSynchronize(s));
        if (err) throw cg::Error(CG_E_DEVICE, "kernel error flag set (look-back bound or offset check)");
        return CG_OK;
    });
}

int cg_test_sort_below(uint64_t *d_keys, uint64_t *d_tmp, uint64_t count, int key_bits, void *stream) {
    return guarded([&]() -> int {
        if (key_bits < 1 || key_bits > 64) throw cg::Error(CG_E_INVAL, "key_bits out of 1..64");
        if (count && (!d_keys || !d_tmp)) throw cg::Error(CG_E_INVAL, "NULL device pointer");
        hipStream_t s = (hipStream_t)stream;
        cg::PipeWork w;
        w.init(s);
        uint64_t *res = cg::radix_sort(d_keys, d_tmp, count, 0, key_bits, w, true);
        if (res != d_keys)
            CG_HIP(hipMemcpyAsync(d_keys, res, count * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        uint32_t err = 0;
        CG_HIP(hipMemcpyAsync(&err, w.err(), sizeof err, hipMemcpyDeviceToHost, s));
        CG_HIP(hipStreamSynchronize(s));
        if (err) throw cg::Error(CG_E_DEVICE, "kernel error flag set (look-back bound or offset check)");
        return CG_OK;
    });
}

int cg_test_sort32(uint32_t *d_keys, uint32_t *d_tmp, uint64_t count, int bit_lo, int bit_hi,
                   void *stream) {
    return guarded([&]() -> int {
        if (bit_lo < 0 || bit_hi > 32 || bit_lo >= bit_hi) throw cg::Error(CG_E_INVAL, "bad bit range");
        if (count && (!d_keys || !d_tmp)) throw cg::Error(CG_E_INVAL, "NULL device pointer");
        hipStream_t s = (hipStream_t)stream;
        cg::PipeWork w;
        w.init(s);
        uint32_t *res = cg::radix_sort32(d_keys, d_tmp, count, bit_lo, bit_hi, w);
        if (res != d_keys)
            CG_HIP(hipMemcpyAsync(d_keys, res, count * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
        uint32_t err = 0;
        CG_HIP(hipMemcpyAsync(&err, w.err(), sizeof err, hipMemcpyDeviceToHost, s));
        CG_HIP(hipStreamSynchronize(s));
        if (err) throw cg::Error(CG_E_DEVICE, "kernel error flag set (look-back bound or offset check)");
        return CG_OK;
    });
}

int cg_test_dedup(const uint64_t *d_sorted, uint64_t C, const uint64_t *d_a, uint64_t na,
                  const uint64_t *d_b, uint64_t nb, uint64_t *d_out, uint64_t *h_count,
                  void *stream) {
    return guarded([&]() -> int {
        if (!h_count || (C && (!d_sorted || !d_out)) || (na && !d_a) || (nb && !d_b))
            throw cg::Error(CG_E_INVAL, "NULL pointer");
        hipStream_t s = (hipStream_t)stream;
        cg::PipeWork w;
        w.init(s);
        cg::DevBuf tmp;
        tmp.stream = s;
        tmp.ensure(C * sizeof(uint64_t) + 8);
        cg::launch_dedup(d_sorted, C, d_a, na, d_b, nb, d_out, C, tmp.as<uint64_t>(), w.counter(), w);
        uint64_t cnt = 0;
        uint32_t err = 0;
        CG_HIP(hipMemcpyAsync(&cnt, w.counter(), sizeof cnt, hipMemcpyDeviceToHost, s));
        CG_HIP(hipMemcpyAsync(&err, w.err(), sizeof err, hipMemcpyDeviceToHost, s));
        CG_HIP(hipStreamSynchronize(s));
        if (err) throw cg::Error(CG_E_DEVICE, "kernel error flag set (look-back bound or offset check)");
        *h_count = cnt;
        return CG_OK;
    });
}

int cg_test_layer_step(int n, const uint8_t *h_gens, int k, const uint64_t *d_frontier, uint64_t F,
                       const uint64_t *d_prev, uint64_t np, uint64_t *d_out, uint64_t *h_count,
                       void *stream) {
    return guarded([&]() -> int {
        auto sels = make_sels(n, h_gens, k);
        if (!h_count || (F && (!d_frontier || !d_out)) || (np && !d_prev))
            throw cg::Error(CG_E_INVAL, "NULL pointer");
        hipStream_t s = (hipStream_t)stream;
        cg::PipeWork w;
        w.init(s);
        cg::DevBuf gs, c0, c1;
        gs.stream = c0.stream = c1.stream = s;
        gs.ensure(sizeof(cg::GenSel) * k);
        CG_HIP(hipMemcpyAsync(gs.p, sels.data(), sizeof(cg::GenSel) * k, hipMemcpyHostToDevice, s));
        const uint64_t C = F * (uint64_t)k;
        c0.ensure(C * 8 + 8);
        c1.ensure(C * 8 + 8);
        const uint64_t *sorted =
            cg::expand_sort(d_frontier, F, gs.as<cg::GenSel>(), k, c0.as<uint64_t>(), c1.as<uint64_t>(),
                            4, 4 * n, w);
        uint64_t *scratch = sorted == c0.as<uint64_t>() ? c1.as<uint64_t>() : c0.as<uint64_t>();
        cg::launch_dedup(sorted, C, d_frontier, F, d_prev, np, d_out, C, scratch, w.counter(), w);
        uint64_t cnt = 0;
        uint32_t err = 0;
        CG_HIP(hipMemcpyAsync(&cnt, w.counter(), sizeof cnt, hipMemcpyDeviceToHost, s));
        CG_HIP(hipMemcpyAsync(&err, w.err(), sizeof err, hipMemcpyDeviceToHost, s));
        CG_HIP(hipStreamSynchronize(s));
        if (err) throw cg::Error(CG_E_DEVICE, "kernel error flag set (look-back bound or offset check)");
        *h_count = cnt;
        return CG_OK;
    });
}

// ---- rank / unrank / host expand -------------------------------------------------

namespace {

// Plain copy, one 16-byte element per lane and one grid over the whole
// array (on MI355X this measured faster than grid-stride loops, with or
// without unrolled or non-temporal accesses): the measured HBM ceiling, and
// the reference for what the traffic counters read for a known byte count.
__global__ __launch_bounds__(256) void copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                   uint64_t n16) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) dst[i] = src[i];
}

// the rank and unrank of the growth kernels (n fixed at compile time)
extern "C++" {
template <int N>
__global__ void rank_kernel(const uint64_t *k, uint64_t count, uint32_t *r) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) r[i] = cg::perm_rank_t<N>(k[i]);
}

template <int N>
__global__ void unrank_kernel(const uint32_t *r, uint64_t count, uint64_t *k) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) k[i] = cg::perm_unrank_t<N>(r[i]);
}

template <int N>
__global__ void rank64_kernel(const uint64_t *k, uint64_t count, uint64_t *r) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) r[i] = cg::perm_rank_t<N, uint64_t>(k[i]);
}

template <int N>
__global__ void unrank64_kernel(const uint64_t *r, uint64_t count, uint64_t *k) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) k[i] = cg::perm_unrank_t<N, uint64_t>(r[i]);
}
}

// v_perm_b32: byte j of the result selects from the 8-byte {s0:s1} (s1 the
// low dword); selector 0x0C gives zero.
uint32_t vperm_host(uint32_t s0, uint32_t s1, uint32_t sel) {
    const uint64_t src = ((uint64_t)s0 << 32) | s1;
    uint32_t out = 0;
    for (int j = 0; j < 4; ++j) {
        const uint32_t b = (sel >> (8 * j)) & 0xFF;
        uint32_t v = 0;
        if (b < 8)
            v = (uint32_t)((src >> (8 * b)) & 0xFF);
        else if (b == 12)
            v = 0;
        else
            v = b >= 13 ? 0xFF : 0;  // sign replication forms are never produced
        out |= v << (8 * j);
    }
    return out;
}

}  // namespace

int cg_test_rank(int n, const uint64_t *h_keys, uint64_t count, uint32_t *h_ranks, int on_device,
                 void *stream) {
    return guarded([&]() -> int {
        if (n < 1 || n > cg::kRankMaxN || (count && (!h_keys || !h_ranks)))
            throw cg::Error(CG_E_INVAL, "bad rank arguments");
        if (!on_device) {
            cg::with_rank_n(n, [&](auto NN) {
                for (uint64_t i = 0; i < count; ++i) h_ranks[i] = cg::perm_rank_t<decltype(NN)::value>(h_keys[i]);
            });
            return CG_OK;
        }
        if (!count) return CG_OK;
        hipStream_t s = (hipStream_t)stream;
        cg::DevBuf a, b;
        a.stream = b.stream = s;
        a.ensure(count * 8);
        b.ensure(count * 4);
        CG_HIP(hipMemcpyAsync(a.p, h_keys, count * 8, hipMemcpyHostToDevice, s));
        cg::with_rank_n(n, [&](auto NN) {
            hipLaunchKernelGGL(rank_kernel<decltype(NN)::value>, dim3((uint32_t)((count + 255) / 256)), dim3(256),
                               0, s, a.as<uint64_t>(), count, b.as<uint32_t>());
        });
        CG_HIP(hipGetLastError());
        CG_HIP(hipMemcpyAsync(h_ranks, b.p, count * 4, hipMemcpyDeviceToHost, s));
        CG_HIP(hipStreamSynchronize(s));
        return CG_OK;
    });
}

int cg_test_unrank(int n, const uint32_t *h_ranks, uint64_t count, uint64_t *h_keys, int on_device,
                   void *stream) {
    return guarded([&]() -> int {
        if (n < 1 || n > cg::kRankMaxN || (count && (!h_keys || !h_ranks)))
            throw cg::Error(CG_E_INVAL, "bad unrank arguments");
        uint64_t fact = 1;
        for (int i = 2; i <= n; ++i) fact *= (uint64_t)i;
        for (uint64_t i = 0; i < count; ++i)
            if (h_ranks[i] >= fact) throw cg::Error(CG_E_INVAL, "rank out of range");
        if (!on_device) {
            cg::with_rank_n(n, [&](auto NN) {
                for (uint64_t i = 0; i < count; ++i) h_keys[i] = cg::perm_unrank_t<decltype(NN)::value>(h_ranks[i]);
            });
            return CG_OK;
        }
        if (!count) return CG_OK;
        hipStream_t s = (hipStream_t)stream;
        cg::DevBuf a, b;
        a.stream = b.stream = s;
        a.ensure(count * 4);
        b.ensure(count * 8);
        CG_HIP(hipMemcpyAsync(a.p, h_ranks, count * 4, hipMemcpyHostToDevice, s));
        cg::with_rank_n(n, [&](auto NN) {
            hipLaunchKernelGGL(unrank_kernel<decltype(NN)::value>, dim3((uint32_t)((count + 255) / 256)),
                               dim3(256), 0, s, a.as<uint32_t>(), count, b.as<uint64_t>());
        });
        CG_HIP(hipGetLastError());
        CG_HIP(hipMemcpyAsync(h_keys, b.p, count * 8, hipMemcpyDeviceToHost, s));
        CG_HIP(hipStreamSynchronize(s));
        return CG_OK;
    });
}

// 64-bit ranks (n = 13..16): the code of the growth kernels, on the host
// or on the device. kind 0 = rank (in: packed keys), 1 = unrank (in: ranks).
static int rank64_impl(int kind, int n, const uint64_t *h_in, uint64_t count, uint64_t *h_out, int on_device,
                       void *stream) {
    return guarded([&]() -> int {
        if (n < cg::kRankMaxN + 1 || n > cg::kRank64MaxN || (count && (!h_in || !h_out)))
            throw cg::Error(CG_E_INVAL, "bad 64-bit rank arguments (n must be 13..16)");
        if (kind == 1) {
            uint64_t fact = 1;
            for (int i = 2; i <= n; ++i) fact *= (uint64_t)i;
            for (uint64_t i = 0; i < count; ++i)
                if (h_in[i] >= fact) throw cg::Error(CG_E_INVAL, "rank out of range");
        }
        if (!on_device) {
            cg::with_rank64_n(n, [&](auto NN) {
                constexpr int N = decltype(NN)::value;
                for (uint64_t i = 0; i < count; ++i)
                    h_out[i] = kind == 0 ? cg::perm_rank_t<N, uint64_t>(h_in[i]) : cg::perm_unrank_t<N, uint64_t>(h_in[i]);
            });
            return CG_OK;
        }
        if (!count) return CG_OK;
        hipStream_t s = (hipStream_t)stream;
        cg::DevBuf a, b;
        a.stream = b.stream = s;
        a.ensure(count * 8);
        b.ensure(count * 8);
        CG_HIP(hipMemcpyAsync(a.p, h_in, count * 8, hipMemcpyHostToDevice, s));
        const dim3 grid((uint32_t)((count + 255) / 256));
        cg::with_rank64_n(n, [&](auto NN) {
            constexpr int N = decltype(NN)::value;
            if (kind == 0)
                hipLaunchKernelGGL(rank64_kernel<N>, grid, dim3(256), 0, s, a.as<uint64_t>(), count, b.as<uint64_t>());
            else
                hipLaunchKernelGGL(unrank64_kernel<N>, grid, dim3(256), 0, s, a.as<uint64_t>(), count,
                                   b.as<uint64_t>());
        });
        CG_HIP(hipGetLastError());
        CG_HIP(hipMemcpyAsync(h_out, b.p, count * 8, hipMemcpyDeviceToHost, s));
        CG_HIP(hipStreamSynchronize(s));
        return CG_OK;
    });
}

int cg_test_rank64(int n, const uint64_t *h_keys, uint64_t count, uint64_t *h_ranks, int on_device, void *stream) {
    return rank64_impl(0, n, h_keys, count, h_ranks, on_device, stream);
}

int cg_test_unrank64(int n, const uint64_t *h_ranks, uint64_t count, uint64_t *h_keys, int on_device,
                     void *stream) {
    return rank64_impl(1, n, h_ranks, count, h_keys, on_device, stream);
}

int cg_test_copy(const void *d_src, void *d_dst, uint64_t bytes, int repeats, void *stream) {
    return guarded([&]() -> int {
        if ((bytes & 15u) || repeats < 0 || (bytes && (!d_src || !d_dst)) ||
            (((uintptr_t)d_src | (uintptr_t)d_dst) & 15u))
            throw cg::Error(CG_E_INVAL, "copy needs 16-byte aligned buffers and a multiple of 16 bytes");
        if (!bytes) return CG_OK;
        hipStream_t s = (hipStream_t)stream;
        const uint64_t n16 = bytes / 16;
        if ((n16 + 255) / 256 > 0x7fffffffull) throw cg::Error(CG_E_INVAL, "copy larger than one grid covers");
        const uint32_t blocks = (uint32_t)((n16 + 255) / 256);
        for (int r = 0; r < repeats; ++r) {
            hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(256), 0, s, (const uint4 *)d_src, (uint4 *)d_dst,
                               n16);
            CG_HIP(hipGetLastError());
        }
        CG_HIP(hipStreamSynchronize(s));
        return CG_OK;
    });
}

int cg_test_host_expand(int n, const uint8_t *h_gens, int k, const uint64_t *h_frontier, uint64_t F,
                        uint64_t *h_out) {
    return guarded([&]() -> int {
        auto sels = make_sels(n, h_gens, k);
        if (F && (!h_frontier || !h_out)) throw cg::Error(CG_E_INVAL, "NULL pointer");
        for (int g = 0; g < k; ++g) {
            const cg::GenSel &sel = sels[g];
            for (uint64_t f = 0; f < F; ++f) {
                const uint64_t key = h_frontier[f];
                const uint32_t lo = (uint32_t)key, hi = (uint32_t)(key >> 32);
                const uint32_t e0 = lo & 0x0F0F0F0Fu, o0 = (lo >> 4) & 0x0F0F0F0Fu;
                const uint32_t e1 = hi & 0x0F0F0F0Fu, o1 = (hi >> 4) & 0x0F0F0F0Fu;
                const uint32_t ye0 = vperm_host(e1, e0, sel.sel[0]) | vperm_host(o1, o0, sel.sel[1]);
                const uint32_t ye1 = vperm_host(e1, e0, sel.sel[2]) | vperm_host(o1, o0, sel.sel[3]);
                const uint32_t yo0 = vperm_host(e1, e0, sel.sel[4]) | vperm_host(o1, o0, sel.sel[5]);
                const uint32_t yo1 = vperm_host(e1, e0, sel.sel[6]) | vperm_host(o1, o0, sel.sel[7]);
                h_out[(uint64_t)g * F + f] = ((uint64_t)(ye1 | (yo1 << 4)) << 32) | (ye0 | (yo0 << 4));
            }
        }
        return CG_OK;
    });
}

int cg_test_host_expand_bits(int n, const uint8_t *h_gens, int k, const uint64_t *h_frontier, uint64_t F,
                             uint64_t *h_out) {
    return guarded([&]() -> int {
        if (n < 1 || n > 64 || k < 1 || !h_gens) throw cg::Error(CG_E_INVAL, "bad generator arguments");
        if (F && (!h_frontier || !h_out)) throw cg::Error(CG_E_INVAL, "NULL pointer");
        for (int g = 0; g < k; ++g) {
            bool seen[64] = {false};
            for (int i = 0; i < n; ++i) {
                const uint8_t v = h_gens[(size_t)g * n + i];
                if (v >= n || seen[v]) throw cg::Error(CG_E_INVAL, "generator row is not a permutation");
                seen[v] = true;
            }
        }
        const std::vector<uint64_t> t = cg::make_bit_tables(n, h_gens, k);
        const int nb = (n + 7) / 8;
        for (int g = 0; g < k; ++g) {
            const uint64_t *tg = t.data() + (size_t)g * nb * 256;
            for (uint64_t f = 0; f < F; ++f) {
                uint64_t x = 0;
                for (int b = 0; b < nb; ++b) x |= tg[b * 256 + ((h_frontier[f] >> (8 * b)) & 255u)];
                h_out[(uint64_t)g * F + f] = x;
            }
        }
        return CG_OK;
    });
}

}  // extern "C"
