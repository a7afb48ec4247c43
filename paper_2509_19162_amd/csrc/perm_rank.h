// Lexicographic rank of a permutation held as a 4-bit-packed key, and its
// inverse. rank(key) = sum_i c_i (n-1-i)!, where c_i counts the values
// smaller than s[i] that do not occur before position i (the Lehmer code);
// it is a bijection from S_n onto [0, n!) that preserves order, so sorting
// ranks sorts the keys. Used for n <= 12 (12! < 2^32) to sort and compare
// candidates as 32-bit words while layers stay packed 64-bit keys.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cg {

constexpr int kRankMaxN = 12;

__host__ __device__ __forceinline__ uint32_t perm_rank(uint64_t key, int n) {
    uint32_t rank = 0, used = 0;
    for (int i = 0; i < n; ++i) {
        const uint32_t v = (uint32_t)(key >> (4 * (n - 1 - i))) & 15u;
        const uint32_t c = v - (uint32_t)__builtin_popcount(used & ((1u << v) - 1u));
        rank = rank * (uint32_t)(n - i) + c;
        used |= 1u << v;
    }
    return rank;
}

__host__ __device__ __forceinline__ uint64_t perm_unrank(uint32_t rank, int n) {
    // mixed-radix digits, last position first
    uint32_t c[16];
    for (int i = n - 1; i >= 0; --i) {
        const uint32_t radix = (uint32_t)(n - i);
        c[i] = rank % radix;
        rank /= radix;
    }
    uint64_t avail = 0;  // nibble j holds the j-th smallest unused value
    for (int j = 0; j < n; ++j) avail |= (uint64_t)j << (4 * j);
    uint64_t key = 0;
    for (int i = 0; i < n; ++i) {
        const uint32_t sh = 4 * c[i];
        const uint64_t v = (avail >> sh) & 15u;
        const uint64_t low = sh ? (avail & ((1ull << sh) - 1ull)) : 0ull;
        avail = low | ((avail >> (sh + 4)) << sh);
        key |= v << (4 * (n - 1 - i));
    }
    return key;
}

}  // namespace cg
