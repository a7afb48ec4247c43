// Kernels of the batched path: many growth jobs advanced together.
//
// A batched key is  (slot << shift) | key(s)  where slot is the job's index
// in its group and shift = 4 * (largest n in the group). Keys of one job
// are contiguous in every sorted array, so one sort, unique, set difference
// and compaction per super-step serve every job of the group, and the tag
// keeps jobs apart (a state of one job never equals a state of another).
#include "batch.h"
#include "device_util.h"
#include "expand_device.h"

namespace cg {

namespace {

// One thread per frontier key: job `slot` (from the tag) expands it by its
// kk[slot] generators into the job's candidate range.
__global__ __launch_bounds__(256) void batch_expand_kernel(
    const uint64_t *__restrict__ frontier, uint64_t total_f, const BatchJobDev *__restrict__ jobs,
    const GenSel *__restrict__ gsel, uint64_t *__restrict__ out, int shift, uint64_t total_c,
    uint32_t nslots, uint32_t *__restrict__ err) {
    const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= total_f) return;
    const uint64_t key = frontier[x];
    const uint32_t slot = shift >= 64 ? 0u : (uint32_t)(key >> shift);
    if (slot >= nslots) {
        atomicOr(err, 8u);
        return;
    }
    const BatchJobDev J = jobs[slot];
    if (J.kk == 0) return;
    const uint64_t tagbits = shift >= 64 ? 0 : ((uint64_t)slot << shift);
    const Nibbles s = split_nibbles(key - tagbits);
    const uint64_t base = J.cand_off + (x - J.front_off) * J.kk;
    if (x < J.front_off || base + J.kk > total_c) {
        atomicOr(err, 8u);  // job table inconsistent with the frontier
        return;
    }
    for (uint32_t g = 0; g < J.kk; ++g) out[base + g] = tagbits | apply_gensel(s, gsel[J.goff + g]);
}

// Per-job sizes of a sorted batched layer: the keys of slot s form one run
// starting at lower_bound(s << shift), so one binary search per slot
// boundary gives every count without reading the layer.
__global__ __launch_bounds__(256) void tag_bounds_kernel(const uint64_t *__restrict__ keys, uint64_t n,
                                                         int shift, uint32_t nslots,
                                                         unsigned long long *__restrict__ pos) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s > nslots) return;
    if (shift >= 64) {
        pos[s] = s == 0 ? 0 : n;
        return;
    }
    const uint64_t key = s >= nslots ? ~0ull : ((uint64_t)s << shift);
    if (s >= nslots) {
        pos[s] = n;
        return;
    }
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (keys[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    pos[s] = lo;
}

__global__ void bounds_to_counts_kernel(const unsigned long long *__restrict__ pos, uint32_t nslots,
                                        unsigned long long *__restrict__ cnt) {
    const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nslots) cnt[s] = pos[s + 1] - pos[s];
}

// Merge of two sorted arrays with no common key: every element lands at its
// own index plus the number of smaller elements of the other array.
__global__ __launch_bounds__(256) void merge_place_kernel(const uint64_t *__restrict__ src, uint64_t n,
                                                          const uint64_t *__restrict__ other, uint64_t m,
                                                          uint64_t *__restrict__ out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t key = src[i];
    uint64_t lo = 0, hi = m;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (other[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    out[i + lo] = key;
}

}  // namespace

void launch_merge(const uint64_t *a, uint64_t na, const uint64_t *b, uint64_t nb, uint64_t *out,
                  hipStream_t s) {
    if (na)
        hipLaunchKernelGGL(merge_place_kernel, dim3((uint32_t)((na + 255) / 256)), dim3(256), 0, s, a, na, b,
                           nb, out);
    CG_HIP(hipGetLastError());
    if (nb)
        hipLaunchKernelGGL(merge_place_kernel, dim3((uint32_t)((nb + 255) / 256)), dim3(256), 0, s, b, nb, a,
                           na, out);
    CG_HIP(hipGetLastError());
}

void launch_batch_expand(const uint64_t *frontier, uint64_t total_f, const BatchJobDev *d_jobs,
                         const GenSel *d_gsel, uint64_t *out, int shift, uint64_t total_c,
                         uint32_t nslots, PipeWork &w) {
    if (!total_f) return;
    if (w.prof) w.prof->begin(K_EXPAND);
    hipLaunchKernelGGL(batch_expand_kernel, dim3((uint32_t)((total_f + 255) / 256)), dim3(256), 0, w.stream,
                       frontier, total_f, d_jobs, d_gsel, out, shift, total_c, nslots, w.err());
    CG_HIP(hipGetLastError());
    if (w.prof) w.prof->end(K_EXPAND, 8.0 * (double)total_f + 8.0 * (double)total_c, (double)total_c);
}

void launch_tag_count(const uint64_t *keys, uint64_t n, int shift, unsigned long long *d_cnt,
                      unsigned long long *d_pos, uint32_t nslots, PipeWork &w) {
    hipLaunchKernelGGL(tag_bounds_kernel, dim3((nslots + 1 + 255) / 256), dim3(256), 0, w.stream, keys, n,
                       shift, nslots, d_pos);
    CG_HIP(hipGetLastError());
    hipLaunchKernelGGL(bounds_to_counts_kernel, dim3((nslots + 255) / 256), dim3(256), 0, w.stream, d_pos,
                       nslots, d_cnt);
    CG_HIP(hipGetLastError());
}

}  // namespace cg
