// Binary states: one bit per entry, for the Schreier coset graphs of a 0/1
// start vector (the central states of the paper's section "Growth of
// Reversals and Transposons on binary cosets", and the coset graphs of
// section "Examples and Tutorials"), n <= 64. Entry i is bit n-1-i of the
// key, so the numeric order of keys is the lexicographic order of the
// vectors, as with the 4-bit packing of permutation states.
//
// The candidate t = s.g (t[i] = s[g[i]], the gather action) is a bit
// permutation of s. For every generator the host builds byte tables:
// T[b][v], for each set bit j of the value v of key byte b (key bit
// p = 8b + j, entry e = n-1-p), holds the candidate bit n-1-i of the one
// position i with g[i] = e. A candidate is then the OR of ceil(n/8) table
// entries, one per key byte. The expand stages one generator's tables in
// LDS at a time and applies it to a round of frontier states held in
// registers.
#include "internal.h"
#include "device_util.h"

namespace cg {

namespace {

constexpr int kBitsBlock = 256;
constexpr int kBitsIpt = 16;                          // frontier states per thread per round
constexpr uint64_t kBitsRound = (uint64_t)kBitsBlock * kBitsIpt;
constexpr int kBitsTable = 256;                       // entries per key byte

__global__ __launch_bounds__(kBitsBlock) void expand_bits_kernel(const uint64_t *__restrict__ frontier, uint64_t F,
                                                                 const uint64_t *__restrict__ tables, int nb, int k,
                                                                 uint64_t *__restrict__ out, uint64_t per_block) {
    __shared__ uint64_t s_t[8 * kBitsTable];  // one generator's tables (up to 8 key bytes)
    const uint32_t tid = threadIdx.x;
    const uint64_t lo = (uint64_t)blockIdx.x * per_block;
    const uint64_t hi = lo + per_block < F ? lo + per_block : F;
    const uint32_t nt = (uint32_t)nb * kBitsTable;
    // every thread runs the same rounds and generators: the barriers below
    // are reached by the whole block
    for (uint64_t base = lo; base < hi; base += kBitsRound) {
        uint64_t s[kBitsIpt];
#pragma unroll
        for (int j = 0; j < kBitsIpt; ++j) {
            const uint64_t f = base + (uint64_t)j * kBitsBlock + tid;
            s[j] = f < hi ? frontier[f] : 0ull;
        }
        for (int g = 0; g < k; ++g) {
            __syncthreads();  // the previous generator's lookups are done
            const uint64_t *tg = tables + (uint64_t)g * nt;
            for (uint32_t i = tid; i < nt; i += kBitsBlock) s_t[i] = tg[i];
            __syncthreads();
            uint64_t *og = out + (uint64_t)g * F;
#pragma unroll
            for (int j = 0; j < kBitsIpt; ++j) {
                const uint64_t f = base + (uint64_t)j * kBitsBlock + tid;
                if (f >= hi) continue;
                uint64_t t = 0;
                for (int b = 0; b < nb; ++b) t |= s_t[b * kBitsTable + (uint32_t)((s[j] >> (8 * b)) & 255u)];
                og[f] = t;
            }
        }
    }
}

// Key-range chunks of binary candidates (see chunk.hip): the counting pass
// and the filtered expand, with the rounds and staged tables above. The
// range of a candidate is its key >> pshift, 12 bits.
__global__ __launch_bounds__(kBitsBlock) void prefix_hist_bits_kernel(const uint64_t *__restrict__ frontier,
                                                                      uint64_t F,
                                                                      const uint64_t *__restrict__ tables, int nb,
                                                                      int k, int pshift, uint64_t per_block,
                                                                      unsigned long long *__restrict__ hist) {
    __shared__ uint64_t s_t[8 * kBitsTable];
    __shared__ uint32_t s_h[kChunkBins];
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < kChunkBins; i += kBitsBlock) s_h[i] = 0;
    __syncthreads();
    const uint64_t lo = (uint64_t)blockIdx.x * per_block;
    const uint64_t hi = lo + per_block < F ? lo + per_block : F;
    const uint32_t nt = (uint32_t)nb * kBitsTable;
    for (uint64_t base = lo; base < hi; base += kBitsRound) {
        uint64_t s[kBitsIpt];
#pragma unroll
        for (int j = 0; j < kBitsIpt; ++j) {
            const uint64_t f = base + (uint64_t)j * kBitsBlock + tid;
            s[j] = f < hi ? frontier[f] : 0ull;
        }
        for (int g = 0; g < k; ++g) {
            __syncthreads();
            const uint64_t *tg = tables + (uint64_t)g * nt;
            for (uint32_t i = tid; i < nt; i += kBitsBlock) s_t[i] = tg[i];
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kBitsIpt; ++j) {
                const uint64_t f = base + (uint64_t)j * kBitsBlock + tid;
                if (f >= hi) continue;
                uint64_t t = 0;
                for (int b = 0; b < nb; ++b) t |= s_t[b * kBitsTable + (uint32_t)((s[j] >> (8 * b)) & 255u)];
                atomicAdd(&s_h[(uint32_t)(t >> pshift) & (kChunkBins - 1)], 1u);
            }
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < kChunkBins; i += kBitsBlock)
        if (s_h[i]) atomicAdd(&hist[i], (unsigned long long)s_h[i]);
}

// Candidates whose range lies in [blo, bhi), appended through a cursor
// (their order does not matter: a sort follows); at most `cap` are
// written, an overrun raises error bit 8.
__global__ __launch_bounds__(kBitsBlock) void expand_filter_bits_kernel(
    const uint64_t *__restrict__ frontier, uint64_t F, const uint64_t *__restrict__ tables, int nb, int k,
    int pshift, uint32_t blo, uint32_t bhi, uint64_t per_block, uint64_t *__restrict__ out, uint64_t cap,
    unsigned long long *cursor, uint32_t *err) {
    __shared__ uint64_t s_t[8 * kBitsTable];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint64_t lo = (uint64_t)blockIdx.x * per_block;
    const uint64_t hi = lo + per_block < F ? lo + per_block : F;
    const uint32_t nt = (uint32_t)nb * kBitsTable;
    for (uint64_t base = lo; base < hi; base += kBitsRound) {
        uint64_t s[kBitsIpt];
#pragma unroll
        for (int j = 0; j < kBitsIpt; ++j) {
            const uint64_t f = base + (uint64_t)j * kBitsBlock + tid;
            s[j] = f < hi ? frontier[f] : 0ull;
        }
        for (int g = 0; g < k; ++g) {
            __syncthreads();
            const uint64_t *tg = tables + (uint64_t)g * nt;
            for (uint32_t i = tid; i < nt; i += kBitsBlock) s_t[i] = tg[i];
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kBitsIpt; ++j) {
                const uint64_t f = base + (uint64_t)j * kBitsBlock + tid;
                uint64_t t = 0;
                for (int b = 0; b < nb; ++b) t |= s_t[b * kBitsTable + (uint32_t)((s[j] >> (8 * b)) & 255u)];
                const uint32_t bin = (uint32_t)(t >> pshift) & (kChunkBins - 1);
                const bool keep = f < hi && bin >= blo && bin < bhi;
                // every lane of the wave takes part in the ballot
                const uint64_t m = __ballot(keep);
                if (!m) continue;
                unsigned long long at = 0;
                if (lane == 0) at = atomicAdd(cursor, (unsigned long long)__popcll(m));
                at = __shfl(at, 0, kWave);
                if (keep) {
                    const uint64_t pos = at + (uint64_t)__popcll(m & ((1ull << lane) - 1ull));
                    if (pos < cap)
                        out[pos] = t;
                    else
                        atomicOr(err, 8u);
                }
            }
        }
    }
}

__global__ void unpack_bits_kernel(int n, const uint64_t *__restrict__ keys, uint64_t count,
                                   uint8_t *__restrict__ rows) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint64_t k = keys[i];
    for (int j = 0; j < n; ++j) rows[i * n + j] = (uint8_t)((k >> (n - 1 - j)) & 1u);
}

}  // namespace

uint64_t pack_bits_host(int n, const uint8_t *s) {
    uint64_t k = 0;
    for (int i = 0; i < n; ++i) k |= (uint64_t)(s[i] & 1u) << (n - 1 - i);
    return k;
}

std::vector<uint64_t> make_bit_tables(int n, const uint8_t *gens, int k) {
    const int nb = (n + 7) / 8;
    std::vector<uint64_t> t((size_t)k * nb * kBitsTable, 0);
    for (int g = 0; g < k; ++g) {
        const uint8_t *row = gens + (size_t)g * n;
        // where each entry of s goes: candidate position i takes entry row[i]
        uint64_t dest[64] = {0};
        for (int i = 0; i < n; ++i) dest[row[i]] = 1ull << (n - 1 - i);
        uint64_t *tg = t.data() + (size_t)g * nb * kBitsTable;
        for (int b = 0; b < nb; ++b)
            for (int v = 0; v < kBitsTable; ++v) {
                uint64_t x = 0;
                for (int j = 0; j < 8; ++j) {
                    const int p = 8 * b + j;  // key bit
                    if (((v >> j) & 1) && p < n) x |= dest[n - 1 - p];
                }
                tg[b * kBitsTable + v] = x;
            }
    }
    return t;
}

void launch_expand_bits(const uint64_t *frontier, uint64_t F, const uint64_t *d_tables, int n, int k,
                        uint64_t *out, PipeWork &w) {
    if (F == 0 || k == 0) return;
    const int nb = (n + 7) / 8;
    const uint64_t rounds = (F + kBitsRound - 1) / kBitsRound;  // whole rounds per block, at most 4096 blocks
    const uint64_t blocks = rounds < 4096 ? rounds : 4096;
    const uint64_t per_block = ((rounds + blocks - 1) / blocks) * kBitsRound;
    const uint32_t grid = (uint32_t)((F + per_block - 1) / per_block);
    if (w.prof) w.prof->begin(K_EXPAND);
    hipLaunchKernelGGL(expand_bits_kernel, dim3(grid), dim3(kBitsBlock), 0, w.stream, frontier, F, d_tables, nb, k,
                       out, per_block);
    CG_HIP(hipGetLastError());
    if (w.prof) w.prof->end(K_EXPAND, 8.0 * (double)F + 16.0 * (double)F * k, (double)F * k);
}

namespace {
// whole rounds per block, at most 4096 blocks
void bits_grid(uint64_t F, uint64_t &per_block, uint32_t &grid) {
    const uint64_t rounds = (F + kBitsRound - 1) / kBitsRound;
    const uint64_t blocks = rounds < 4096 ? rounds : 4096;
    per_block = ((rounds + blocks - 1) / blocks) * kBitsRound;
    grid = (uint32_t)((F + per_block - 1) / per_block);
}
}  // namespace

void launch_prefix_hist_bits(const uint64_t *frontier, uint64_t F, const uint64_t *d_tables, int n, int k,
                             int pshift, unsigned long long *d_hist, PipeWork &w) {
    if (!F || !k) return;
    uint64_t per_block;
    uint32_t grid;
    bits_grid(F, per_block, grid);
    hipLaunchKernelGGL(prefix_hist_bits_kernel, dim3(grid), dim3(kBitsBlock), 0, w.stream, frontier, F, d_tables,
                       (n + 7) / 8, k, pshift, per_block, d_hist);
    CG_HIP(hipGetLastError());
}

void launch_expand_filter_bits(const uint64_t *frontier, uint64_t F, const uint64_t *d_tables, int n, int k,
                               int pshift, uint32_t blo, uint32_t bhi, uint64_t *out, uint64_t cap,
                               unsigned long long *cursor, PipeWork &w) {
    if (!F || !k) return;
    uint64_t per_block;
    uint32_t grid;
    bits_grid(F, per_block, grid);
    hipLaunchKernelGGL(expand_filter_bits_kernel, dim3(grid), dim3(kBitsBlock), 0, w.stream, frontier, F, d_tables,
                       (n + 7) / 8, k, pshift, blo, bhi, per_block, out, cap, cursor, w.err());
    CG_HIP(hipGetLastError());
}

void launch_unpack_bits(int n, const uint64_t *d_keys, uint64_t count, uint8_t *d_rows, hipStream_t s) {
    if (!count) return;
    hipLaunchKernelGGL(unpack_bits_kernel, dim3((uint32_t)((count + 255) / 256)), dim3(256), 0, s, n, d_keys,
                       count, d_rows);
    CG_HIP(hipGetLastError());
}

}  // namespace cg
