// Permute-expand: every state of the frontier is mapped through every
// generator (paper, section "Reminder on Cayley graphs, diameters, growth":
// an edge joins v and M_k v for every move M_k; the moves are permutations
// of the entries, section "Examples and Tutorials"). Gather convention:
// t[i] = s[g[i]].
//
// A state key holds 16 nibbles. Splitting it into its even and its odd
// nibbles gives 16 bytes, one entry each; a nibble permutation is then a
// byte permutation, which v_perm_b32 does four bytes at a time from an
// 8-byte source. Each output dword takes one v_perm over the even-nibble
// bytes and one over the odd-nibble bytes (selector 0x0C yields a zero
// byte), so one candidate costs 8 v_perm, 4 ORs and 2 shift/OR pairs,
// independent of the generator.
#include "internal.h"
#include "device_util.h"
#include "expand_device.h"
#include "perm_rank.h"

namespace cg {

uint64_t pack_host(int n, const uint8_t *s) {
    uint64_t k = 0;
    for (int i = 0; i < n; ++i) k |= (uint64_t)(s[i] & 15u) << (4 * (n - 1 - i));
    return k;
}

void unpack_host(int n, uint64_t key, uint8_t *s) {
    for (int i = 0; i < n; ++i) s[i] = (uint8_t)((key >> (4 * (n - 1 - i))) & 15u);
}

// Output nibble q (bits 4q..4q+3) is the state's entry at position n-1-q.
// It takes the source nibble qs = n-1-g[n-1-q]. Even source nibbles live in
// the "E" bytes (byte qs/2 of {E1:E0}); odd ones in the "O" bytes (byte
// (qs-1)/2 of {O1:O0}). Output dwords: YE0 = nibbles 0,2,4,6; YE1 = 8..14;
// YO0 = 1,3,5,7; YO1 = 9..15; each assembled as perm(E) | perm(O).
GenSel make_gensel(int n, const uint8_t *g) {
    uint8_t se[16], so[16];
    for (int q = 0; q < 16; ++q) {
        se[q] = so[q] = 0x0C;  // v_perm selector for a zero byte
        if (q < n) {
            const int qs = n - 1 - g[n - 1 - q];
            if ((qs & 1) == 0)
                se[q] = (uint8_t)(qs / 2);
            else
                so[q] = (uint8_t)((qs - 1) / 2);
        }
    }
    auto word = [](const uint8_t *sel, int q0) {
        uint32_t w = 0;
        for (int j = 0; j < 4; ++j) w |= (uint32_t)sel[q0 + 2 * j] << (8 * j);
        return w;
    };
    GenSel r;
    r.sel[0] = word(se, 0);
    r.sel[1] = word(so, 0);
    r.sel[2] = word(se, 8);
    r.sel[3] = word(so, 8);
    r.sel[4] = word(se, 1);
    r.sel[5] = word(so, 1);
    r.sel[6] = word(se, 9);
    r.sel[7] = word(so, 9);
    return r;
}

namespace {

constexpr int kExpandBlock = 256;

// Generator-major output: out[g*F + f]. Each block handles a contiguous
// range of frontier states for one generator, so the selectors are
// wave-uniform (scalar loads) and both the load and the store are
// consecutive 8-byte words across the wave.
__global__ __launch_bounds__(kExpandBlock) void expand_kernel(
    const uint64_t *__restrict__ frontier, uint64_t F, const GenSel *__restrict__ gsel,
    uint64_t *__restrict__ out, uint32_t blocks_per_gen) {
    const uint32_t g = blockIdx.x / blocks_per_gen;
    const uint64_t b = blockIdx.x - (uint64_t)g * blocks_per_gen;
    const GenSel sel = gsel[g];
    const uint64_t stride = (uint64_t)blocks_per_gen * kExpandBlock;
    for (uint64_t f = b * kExpandBlock + threadIdx.x; f < F; f += stride) {
        out[(uint64_t)g * F + f] = apply_gensel(frontier[f], sel);
    }
}

// Same tiling as expand_kernel; each candidate is stored as its 32-bit
// lexicographic rank.
__global__ __launch_bounds__(kExpandBlock) void expand_rank_kernel(
    const uint64_t *__restrict__ frontier, uint64_t F, const GenSel *__restrict__ gsel,
    uint32_t *__restrict__ out, uint32_t blocks_per_gen, int n) {
    const uint32_t g = blockIdx.x / blocks_per_gen;
    const uint64_t b = blockIdx.x - (uint64_t)g * blocks_per_gen;
    const GenSel sel = gsel[g];
    const uint64_t stride = (uint64_t)blocks_per_gen * kExpandBlock;
    for (uint64_t f = b * kExpandBlock + threadIdx.x; f < F; f += stride)
        out[(uint64_t)g * F + f] = perm_rank(apply_gensel(frontier[f], sel), n);
}

__global__ void pack_kernel(int n, const uint8_t *__restrict__ rows, uint64_t count,
                            uint64_t *__restrict__ keys) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    uint64_t k = 0;
    for (int j = 0; j < n; ++j) k |= (uint64_t)(rows[i * n + j] & 15u) << (4 * (n - 1 - j));
    keys[i] = k;
}

__global__ void unpack_kernel(int n, const uint64_t *__restrict__ keys, uint64_t count,
                              uint8_t *__restrict__ rows) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint64_t k = keys[i];
    for (int j = 0; j < n; ++j) rows[i * n + j] = (uint8_t)((k >> (4 * (n - 1 - j))) & 15u);
}

}  // namespace

void launch_expand(const uint64_t *frontier, uint64_t F, const GenSel *d_gsel, int k,
                   uint64_t *out, PipeWork &w) {
    if (F == 0 || k == 0) return;
    // enough blocks per generator to fill the chip, capped so each thread
    // handles a few states
    uint64_t per = (F + kExpandBlock - 1) / kExpandBlock;
    uint64_t want = (2048 + (uint64_t)k - 1) / (uint64_t)k;
    if (want < 8) want = 8;
    uint32_t bpg = (uint32_t)(per < want ? per : want);
    if (bpg == 0) bpg = 1;
    if (w.prof) w.prof->begin(K_EXPAND);
    hipLaunchKernelGGL(expand_kernel, dim3(bpg * (uint32_t)k), dim3(kExpandBlock), 0, w.stream,
                       frontier, F, d_gsel, out, bpg);
    CG_HIP(hipGetLastError());
    if (w.prof) w.prof->end(K_EXPAND, 8.0 * (double)F * k + 8.0 * (double)F, (double)F * k);
}

void launch_expand_ranked(int n, const uint64_t *frontier, uint64_t F, const GenSel *d_gsel, int k,
                          uint32_t *out, PipeWork &w) {
    if (F == 0 || k == 0) return;
    uint64_t per = (F + kExpandBlock - 1) / kExpandBlock;
    uint64_t want = (2048 + (uint64_t)k - 1) / (uint64_t)k;
    if (want < 8) want = 8;
    uint32_t bpg = (uint32_t)(per < want ? per : want);
    if (bpg == 0) bpg = 1;
    if (w.prof) w.prof->begin(K_EXPAND);
    hipLaunchKernelGGL(expand_rank_kernel, dim3(bpg * (uint32_t)k), dim3(kExpandBlock), 0, w.stream,
                       frontier, F, d_gsel, out, bpg, n);
    CG_HIP(hipGetLastError());
    if (w.prof) w.prof->end(K_EXPAND, 4.0 * (double)F * k + 8.0 * (double)F, (double)F * k);
}

void launch_pack(int n, const uint8_t *d_rows, uint64_t count, uint64_t *d_keys,
                 hipStream_t s) {
    if (!count) return;
    hipLaunchKernelGGL(pack_kernel, dim3((uint32_t)((count + 255) / 256)), dim3(256), 0, s, n,
                       d_rows, count, d_keys);
    CG_HIP(hipGetLastError());
}

void launch_unpack(int n, const uint64_t *d_keys, uint64_t count, uint8_t *d_rows,
                   hipStream_t s) {
    if (!count) return;
    hipLaunchKernelGGL(unpack_kernel, dim3((uint32_t)((count + 255) / 256)), dim3(256), 0, s, n,
                       d_keys, count, d_rows);
    CG_HIP(hipGetLastError());
}

}  // namespace cg
