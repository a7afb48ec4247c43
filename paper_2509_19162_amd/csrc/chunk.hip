// Key-range chunks of one layer's candidates, for layers whose candidate
// arrays do not fit in device memory. The candidates' sort keys (32-bit
// ranks, or packed keys on bits [4, 4n)) are split by their top 12 bits:
// a counting pass sizes every range, consecutive ranges are grouped into
// chunks that fit, and each chunk regenerates the candidates from the
// frontier, keeps the ones in its range, and runs the usual sort, unique,
// set difference and compaction. Chunks go in increasing key order, so the
// concatenated survivors are the sorted layer.
#include "internal.h"
#include "device_util.h"
#include "expand_device.h"
#include "perm_rank.h"

namespace cg {

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kBins = kChunkBins;

template <int N, bool Ranked>
__device__ __forceinline__ uint64_t sort_value(uint64_t key) {
    if constexpr (Ranked)
        return (uint64_t)perm_rank_t<N>(key);
    else
        return key;
}

template <int N, bool Ranked>
__global__ __launch_bounds__(kBlock) void prefix_hist_kernel(const uint64_t *__restrict__ frontier, uint64_t F,
                                                             const GenSel *__restrict__ gsel, int k, int pshift,
                                                             unsigned long long *__restrict__ hist) {
    __shared__ uint32_t s_h[kBins];
    for (uint32_t i = threadIdx.x; i < kBins; i += kBlock) s_h[i] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t f = (uint64_t)blockIdx.x * kBlock + threadIdx.x; f < F; f += stride) {
        const Nibbles s = split_nibbles(frontier[f]);
        for (int g = 0; g < k; ++g) {
            const uint64_t v = sort_value<N, Ranked>(apply_gensel(s, gsel[g]));
            atomicAdd(&s_h[(uint32_t)(v >> pshift) & (kBins - 1)], 1u);
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < kBins; i += kBlock)
        if (s_h[i]) atomicAdd(&hist[i], (unsigned long long)s_h[i]);
}

// Candidates whose range index lies in [blo, bhi), appended through a
// cursor (order does not matter: a sort follows). At most `cap` are
// written; an overrun raises error bit 8.
template <int N, bool Ranked, class K>
__global__ __launch_bounds__(kBlock) void expand_filter_kernel(const uint64_t *__restrict__ frontier, uint64_t F,
                                                               const GenSel *__restrict__ gsel, int k, int pshift,
                                                               uint32_t blo, uint32_t bhi, K *__restrict__ out,
                                                               uint64_t cap, unsigned long long *cursor,
                                                               uint32_t *err) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const uint32_t lane = lane_id();
    // every lane of a wave runs the same number of rounds (ballots below)
    for (uint64_t base = (uint64_t)blockIdx.x * kBlock; base < F; base += stride) {
        const uint64_t f = base + threadIdx.x;
        const bool valid = f < F;
        const Nibbles s = split_nibbles(valid ? frontier[f] : 0ull);
        for (int g = 0; g < k; ++g) {
            const uint64_t v = sort_value<N, Ranked>(apply_gensel(s, gsel[g]));
            const uint32_t bin = (uint32_t)(v >> pshift) & (kBins - 1);
            const bool keep = valid && bin >= blo && bin < bhi;
            const uint64_t m = __ballot(keep);
            if (!m) continue;
            unsigned long long at = 0;
            if (lane == 0) at = atomicAdd(cursor, (unsigned long long)__popcll(m));
            at = __shfl(at, 0, kWave);
            if (keep) {
                const uint64_t pos = at + mask_rank(m);
                if (pos < cap)
                    out[pos] = (K)v;
                else
                    atomicOr(err, 8u);
            }
        }
    }
}

uint32_t grid_for(uint64_t F) {
    const uint64_t b = (F + kBlock - 1) / kBlock;
    return (uint32_t)(b < 4096 ? (b ? b : 1) : 4096);
}

}  // namespace

void launch_prefix_hist(int n, bool ranked, const uint64_t *frontier, uint64_t F, const GenSel *d_gsel, int k,
                        int pshift, unsigned long long *d_hist, PipeWork &w) {
    if (!F || !k) return;
    const uint32_t grid = grid_for(F);
    if (ranked) {
        with_rank_n(n, [&](auto NN) {
            hipLaunchKernelGGL((prefix_hist_kernel<decltype(NN)::value, true>), dim3(grid), dim3(kBlock), 0, w.stream,
                               frontier, F, d_gsel, k, pshift, d_hist);
        });
    } else {
        hipLaunchKernelGGL((prefix_hist_kernel<0, false>), dim3(grid), dim3(kBlock), 0, w.stream, frontier, F, d_gsel,
                           k, pshift, d_hist);
    }
    CG_HIP(hipGetLastError());
}

void launch_expand_filter(int n, bool ranked, const uint64_t *frontier, uint64_t F, const GenSel *d_gsel, int k,
                          int pshift, uint32_t blo, uint32_t bhi, void *out, uint64_t cap,
                          unsigned long long *cursor, PipeWork &w) {
    if (!F || !k) return;
    const uint32_t grid = grid_for(F);
    if (ranked) {
        with_rank_n(n, [&](auto NN) {
            hipLaunchKernelGGL((expand_filter_kernel<decltype(NN)::value, true, uint32_t>), dim3(grid), dim3(kBlock),
                               0, w.stream, frontier, F, d_gsel, k, pshift, blo, bhi, (uint32_t *)out, cap, cursor,
                               w.err());
        });
    } else {
        hipLaunchKernelGGL((expand_filter_kernel<0, false, uint64_t>), dim3(grid), dim3(kBlock), 0, w.stream,
                           frontier, F, d_gsel, k, pshift, blo, bhi, (uint64_t *)out, cap, cursor, w.err());
    }
    CG_HIP(hipGetLastError());
}

}  // namespace cg
