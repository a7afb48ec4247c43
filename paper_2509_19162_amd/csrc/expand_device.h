// Device side of the permute-expand step (used by the stand-alone expand
// kernel and by the first sort pass, which regenerates candidates from the
// frontier instead of reading them back).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace cg {

// Split a key into its even nibbles (E, bytes = nibbles 0,2,..,14) and odd
// nibbles (O, bytes = nibbles 1,3,..,15), one entry per byte.
struct Nibbles {
    uint32_t e0, e1, o0, o1;
};

__device__ __forceinline__ Nibbles split_nibbles(uint64_t key) {
    const uint32_t lo = (uint32_t)key, hi = (uint32_t)(key >> 32);
    Nibbles r;
    r.e0 = lo & 0x0F0F0F0Fu;
    r.o0 = (lo >> 4) & 0x0F0F0F0Fu;
    r.e1 = hi & 0x0F0F0F0Fu;
    r.o1 = (hi >> 4) & 0x0F0F0F0Fu;
    return r;
}

// Key of s.g for the generator whose selectors are `g` (make_gensel).
__device__ __forceinline__ uint64_t apply_gensel(const Nibbles &s, const GenSel &g) {
    const uint32_t ye0 = __builtin_amdgcn_perm(s.e1, s.e0, g.sel[0]) |
                         __builtin_amdgcn_perm(s.o1, s.o0, g.sel[1]);
    const uint32_t ye1 = __builtin_amdgcn_perm(s.e1, s.e0, g.sel[2]) |
                         __builtin_amdgcn_perm(s.o1, s.o0, g.sel[3]);
    const uint32_t yo0 = __builtin_amdgcn_perm(s.e1, s.e0, g.sel[4]) |
                         __builtin_amdgcn_perm(s.o1, s.o0, g.sel[5]);
    const uint32_t yo1 = __builtin_amdgcn_perm(s.e1, s.e0, g.sel[6]) |
                         __builtin_amdgcn_perm(s.o1, s.o0, g.sel[7]);
    const uint32_t lo = ye0 | (yo0 << 4);
    const uint32_t hi = ye1 | (yo1 << 4);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t apply_gensel(uint64_t key, const GenSel &g) {
    return apply_gensel(split_nibbles(key), g);
}

}  // namespace cg
