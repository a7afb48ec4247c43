// Lexicographic rank of a permutation held as a 4-bit-packed key, and its
// inverse. rank(key) = sum_i c_i (n-1-i)!, where c_i counts the values
// smaller than s[i] that do not occur before position i (the Lehmer code);
// it is a bijection from S_n onto [0, n!) that preserves order, so sorting
// ranks sorts the keys. Used for n <= 12 (12! < 2^32) to sort and compare
// candidates as 32-bit words while layers stay packed 64-bit keys, and as
// the bit index of the rank-space bitmaps.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace cg {

constexpr int kRankMaxN = 12;    // 32-bit ranks
constexpr int kRank64MaxN = 16;  // 64-bit ranks (16! < 2^45)

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

// a * b + c for a, b < 2^24 (both factors of every use below are): a 24-bit
// multiply-add for 32-bit ranks, a plain one for 64-bit ranks (the product
// may exceed 32 bits there). On the device b goes through a scalar
// register, so it must be the same in every lane (every use passes a
// radix or factorial fixed at compile time).
template <class R>
__host__ __device__ __forceinline__ R mad24(R a, R b, R c) {
#ifdef __HIP_DEVICE_COMPILE__
    if constexpr (sizeof(R) == 4) {
        // written out: left to itself the compiler reassociates the Horner
        // chain into 32-bit multiplies (quarter rate)
        uint32_t r;
        __asm__("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"((uint32_t)a), "s"((uint32_t)b), "v"((uint32_t)c));
        return (R)r;
    }
#endif
    return a * b + c;
}

// The low v bits of x (v < 32): on the device one bit-field extract, where
// the plain expression costs a mask build and an AND.
__host__ __device__ __forceinline__ uint32_t low_bits(uint32_t x, uint32_t v) {
#ifdef __HIP_DEVICE_COMPILE__
    return __builtin_amdgcn_ubfe(x, 0u, v);
#else
    return x & ((1u << v) - 1u);
#endif
}

// Last position whose Horner prefix N (N-1) ... (N-i) stays below 2^24.
template <int N>
constexpr int rank_split() {
    uint64_t bound = (uint64_t)N;
    int i = 0;
    while (i + 1 < N - 1 && bound * (uint64_t)(N - i - 1) < (1ull << 24)) {
        bound *= (uint64_t)(N - i - 1);
        ++i;
    }
    return i;
}

// Radix of the low part of the split Horner sum: the product of the radices
// N-i of positions kHi+1 .. N-2, i.e. (N-1-kHi)!. It stays below 2^24 for
// every N <= 16 (16: 10! = 3628800), so the low part is 24-bit work too.
template <int N>
constexpr uint32_t rank_lo_radix() {
    uint32_t r = 1;
    for (int i = rank_split<N>() + 1; i < N - 1; ++i) r *= (uint32_t)(N - i);
    return r;
}

// The same with n fixed at compile time: the loops unroll, shifts become
// constants and the divisions of the unrank become multiplications. R is
// the rank type: uint32_t up to n = 12, uint64_t beyond (16! < 2^45).
template <int N, class R = uint32_t>
__host__ __device__ __forceinline__ R perm_rank_t(uint64_t key) {
    // c_i = number of values below s[i] not used before position i: the
    // popcount of the low s[i] bits of the still-unused set. The first
    // position has c_0 = s[0]; the last always has c = 0.
    //
    // The Horner sum is split in two: positions 0..kHi accumulate in `hi`,
    // whose bound N (N-1) ... (N-kHi) stays below 2^24, the rest in `lo`
    // (below rank_lo_radix<N>() < 2^24); rank = hi * lo_radix + lo. Every
    // step is then a 24-bit multiply-add (full rate) instead of a 32- or
    // 64-bit multiply; a 64-bit rank takes one 64-bit multiply-add at the
    // end.
    if constexpr (N <= 1) {
        return 0;
    } else {
        constexpr int kHi = rank_split<N>();
        constexpr uint32_t kLoRadix = rank_lo_radix<N>();
        static_assert(kLoRadix < (1u << 24), "low part of the rank in 24 bits");
        static_assert(sizeof(R) == 8 || N <= 12, "32-bit ranks up to n = 12");
        uint32_t unused = (1u << N) - 1u;
        const uint32_t v0 = (uint32_t)(key >> (4 * (N - 1))) & 15u;
        uint32_t hi = v0, lo = 0;
        unused ^= 1u << v0;
#pragma unroll
        for (int i = 1; i < N - 1; ++i) {
            const uint32_t v = (uint32_t)(key >> (4 * (N - 1 - i))) & 15u;
            const uint32_t c = (uint32_t)__builtin_popcount(low_bits(unused, v));
            if (i <= kHi)
                hi = mad24<uint32_t>(hi, (uint32_t)(N - i), c);
            else
                lo = mad24<uint32_t>(lo, (uint32_t)(N - i), c);
            unused ^= 1u << v;
        }
        // the last position's digit is 0 (radix 1)
        if constexpr (sizeof(R) == 4)
            return mad24<uint32_t>(hi, kLoRadix, lo);
        else
            return (uint64_t)hi * (uint64_t)kLoRadix + (uint64_t)lo;
    }
}

// The inverse with n fixed at compile time (n <= 16). The unused values,
// smallest first, are kept as a list of nibbles in two 32-bit words (lo:
// entries 0-7, hi: entries 8-15), so every step is 32-bit work: read entry
// c, then move the entries after it down one nibble, from hi into lo where
// the list still reaches into hi (decided at compile time per position).
// A 64-bit rank is split once, by one division by rank_lo_radix<N>(), into
// two parts below 2^24 whose digits come from 32-bit divisions.
template <int N, class R = uint32_t>
__host__ __device__ __forceinline__ uint64_t perm_unrank_t(R rank) {
    static_assert(N <= 16, "16 nibbles at most");
    uint32_t c[N > 0 ? N : 1];
    if constexpr (sizeof(R) == 8 && N > 1) {
        constexpr int kHi = rank_split<N>();
        constexpr uint64_t kLoRadix = rank_lo_radix<N>();
        const uint64_t q = rank / kLoRadix;
        uint32_t lo = (uint32_t)(rank - q * kLoRadix), hi = (uint32_t)q;
#pragma unroll
        for (int i = N - 1; i > kHi; --i) {
            c[i] = lo % (uint32_t)(N - i);
            lo /= (uint32_t)(N - i);
        }
#pragma unroll
        for (int i = kHi; i >= 0; --i) {
            c[i] = hi % (uint32_t)(N - i);
            hi /= (uint32_t)(N - i);
        }
    } else {
#pragma unroll
        for (int i = N - 1; i >= 0; --i) {
            c[i] = (uint32_t)(rank % (R)(N - i));
            rank /= (R)(N - i);
        }
    }
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if (j < 8)
            lo |= (uint32_t)j << (4 * j);
        else
            hi |= (uint32_t)j << (4 * (j - 8));
    }
    uint32_t klo = 0, khi = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const uint32_t sh = 4 * c[i];  // c[i] < N - i
        uint32_t v;
        if (N - i > 8) {
            const bool in_hi = sh >= 32u;
            const uint32_t s5 = sh & 31u;
            v = ((in_hi ? hi : lo) >> s5) & 15u;
            const uint32_t keep = (1u << s5) - 1u;  // the entries before c stay
            const uint32_t lo_dn = (lo >> 4) | (hi << 28);
            const uint32_t hi_dn = hi >> 4;
            const uint32_t lo_rm = (lo & keep) | (lo_dn & ~keep);
            const uint32_t hi_rm = (hi & keep) | (hi_dn & ~keep);
            lo = in_hi ? lo : lo_rm;
            hi = in_hi ? hi_rm : hi_dn;
        } else {  // at most 8 entries left, all in lo
            v = (lo >> sh) & 15u;
            const uint32_t keep = (1u << sh) - 1u;
            lo = (lo & keep) | ((lo >> 4) & ~keep);
        }
        const int pos = 4 * (N - 1 - i);
        if (pos >= 32)
            khi |= v << (pos - 32);
        else
            klo |= v << pos;
    }
    return ((uint64_t)khi << 32) | klo;
}

// Calls f(std::integral_constant<int, N>{}) for the runtime n in 13..16:
// the groups whose ranks need 64 bits (13! > 2^32).
template <class F>
void with_rank64_n(int n, F &&f) {
    switch (n) {
        case 13: f(std::integral_constant<int, 13>{}); break;
        case 14: f(std::integral_constant<int, 14>{}); break;
        case 15: f(std::integral_constant<int, 15>{}); break;
        default: f(std::integral_constant<int, 16>{}); break;
    }
}

// Calls f(std::integral_constant<int, N>{}) for the runtime n in 1..12.
template <class F>
void with_rank_n(int n, F &&f) {
    switch (n) {
        case 1: f(std::integral_constant<int, 1>{}); break;
        case 2: f(std::integral_constant<int, 2>{}); break;
        case 3: f(std::integral_constant<int, 3>{}); break;
        case 4: f(std::integral_constant<int, 4>{}); break;
        case 5: f(std::integral_constant<int, 5>{}); break;
        case 6: f(std::integral_constant<int, 6>{}); break;
        case 7: f(std::integral_constant<int, 7>{}); break;
        case 8: f(std::integral_constant<int, 8>{}); break;
        case 9: f(std::integral_constant<int, 9>{}); break;
        case 10: f(std::integral_constant<int, 10>{}); break;
        case 11: f(std::integral_constant<int, 11>{}); break;
        default: f(std::integral_constant<int, 12>{}); break;
    }
}

}  // namespace cg
