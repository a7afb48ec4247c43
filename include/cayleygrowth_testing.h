/*
 * cayleygrowth_testing.h -- kernel-level entry points of libcayleygrowth.so.
 *
 * Each call runs ONE stage of the breadth-first growth step on device
 * buffers the caller owns (for example tensors allocated by PyTorch), so
 * that tests can check every stage against a CPU reference on its own.
 * The stages are the steps of one layer of the search (paper, section
 * "Reminder on Cayley graphs, diameters, growth", definition of Growth;
 * the search is the breadth-first one the section "Examples and Tutorials"
 * names): expand every state by every generator, sort, drop repeats and
 * states of the two previous layers, compact.
 *
 * State keys: a state s with n <= 16 entries is the uint64
 *     key(s) = sum_i s[i] << 4*(n-1-i)
 * (entry 0 in the most significant used nibble, unused high nibbles zero),
 * so numeric order of keys is lexicographic order of states.
 *
 * Pointers named d_* are device pointers; h_* are host pointers. All calls
 * are enqueued on `stream` (a hipStream_t, NULL = the null stream) and
 * synchronise it before returning. Return CG_OK or a negative CG_E_* code.
 */
#ifndef CAYLEYGROWTH_TESTING_H
#define CAYLEYGROWTH_TESTING_H

#include "cayleygrowth.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Pack n-byte rows (host) into keys (device). h_states: count*n bytes. */
int cg_test_pack(int n, const uint8_t *h_states, uint64_t count,
                 uint64_t *d_keys, void *stream);

/* Unpack keys (device) into n-byte rows (host). */
int cg_test_unpack(int n, const uint64_t *d_keys, uint64_t count,
                   uint8_t *h_states, void *stream);

/*
 * Permute-expand: d_out[g*F + f] = key(s_f . g) for every frontier key
 * d_frontier[f] (f < F) and every generator row g (< k) of h_gens (k rows
 * of n bytes, each a permutation of 0..n-1). d_out holds k*F keys.
 */
int cg_test_expand(int n, const uint8_t *h_gens, int k,
                   const uint64_t *d_frontier, uint64_t F, uint64_t *d_out,
                   void *stream);

/*
 * Stable LSD radix sort of d_keys[0..count) on key bits [bit_lo, bit_hi)
 * (0 <= bit_lo < bit_hi <= 64); the result is left in d_keys. d_tmp is a
 * device buffer of count keys used as the second buffer.
 */
int cg_test_sort(uint64_t *d_keys, uint64_t *d_tmp, uint64_t count,
                 int bit_lo, int bit_hi, void *stream);

/*
 * Stable sort of d_keys[0..count) on bits [0, key_bits) (1 <= key_bits <=
 * 64) in digits of balanced widths (45 bits: 7,7,7,8,8,8): the sort the
 * growth step runs on 64-bit lexicographic ranks (n = 13..16) and on binary
 * states, whose keys are all below 2^key_bits. The result is left in
 * d_keys; d_tmp holds count keys.
 */
int cg_test_sort_below(uint64_t *d_keys, uint64_t *d_tmp, uint64_t count,
                       int key_bits, void *stream);

/*
 * The same for 32-bit keys (0 <= bit_lo < bit_hi <= 32): the sort the
 * growth step runs on the lexicographic ranks of candidates for n <= 12,
 * with its own tile shape. d_tmp holds count keys.
 */
int cg_test_sort32(uint32_t *d_keys, uint32_t *d_tmp, uint64_t count,
                   int bit_lo, int bit_hi, void *stream);

/*
 * Unique + set difference + compaction: from the sorted d_sorted[0..C)
 * keep each key once, and only if it is in neither sorted array d_a[0..na)
 * nor d_b[0..nb). The kept keys go to d_out in increasing order;
 * *h_count receives their number. d_out must hold C keys.
 */
int cg_test_dedup(const uint64_t *d_sorted, uint64_t C, const uint64_t *d_a,
                  uint64_t na, const uint64_t *d_b, uint64_t nb,
                  uint64_t *d_out, uint64_t *h_count, void *stream);

/*
 * One full layer step: expand d_frontier (F keys, sorted) by the k
 * generators, sort, drop repeats and keys of d_frontier and d_prev (np
 * keys, sorted), compact into d_out (capacity k*F). *h_count receives the
 * new layer's size. This is exactly the sequence cg_growth runs per layer.
 */
int cg_test_layer_step(int n, const uint8_t *h_gens, int k,
                       const uint64_t *d_frontier, uint64_t F,
                       const uint64_t *d_prev, uint64_t np, uint64_t *d_out,
                       uint64_t *h_count, void *stream);

/*
 * Lexicographic rank of permutation keys (n <= 12): h_ranks[i] = the index
 * of the permutation in lexicographic order of S_n, computed by the rank of
 * the growth kernels (n fixed at compile time). on_device = 1 runs the
 * device code (host buffers are staged), 0 the same code on the host.
 * cg_test_unrank is the inverse (h_ranks < n! required).
 */
int cg_test_rank(int n, const uint64_t *h_keys, uint64_t count, uint32_t *h_ranks,
                 int on_device, void *stream);
int cg_test_unrank(int n, const uint32_t *h_ranks, uint64_t count, uint64_t *h_keys,
                   int on_device, void *stream);

/*
 * The same with 64-bit ranks, for n = 13..16 (16! < 2^45): the rank and
 * unrank that the growth kernels use when candidates of such permutations
 * are sorted and compared as lexicographic ranks. CG_E_INVAL for n outside
 * 13..16 or (unrank) a rank >= n!.
 */
int cg_test_rank64(int n, const uint64_t *h_keys, uint64_t count, uint64_t *h_ranks,
                   int on_device, void *stream);
int cg_test_unrank64(int n, const uint64_t *h_ranks, uint64_t count, uint64_t *h_keys,
                     int on_device, void *stream);

/*
 * Plain device-to-device copy of `bytes` bytes (a multiple of 16, both
 * pointers 16-byte aligned), run `repeats` times. Not part of the method:
 * the known byte count calibrates hardware traffic counters against the
 * kernels of the growth step.
 */
int cg_test_copy(const void *d_src, void *d_dst, uint64_t bytes, int repeats, void *stream);

/*
 * Host emulation of the byte-permute expand (v_perm_b32 semantics written
 * out on the CPU): h_out[g*F + f] = key(s_f . g). Checks the selector
 * tables without a GPU.
 */
int cg_test_host_expand(int n, const uint8_t *h_gens, int k, const uint64_t *h_frontier,
                        uint64_t F, uint64_t *h_out);

/*
 * The expand of binary states (one bit per entry, entry i at bit n-1-i,
 * n <= 64) applied on the host with the byte tables the GPU kernel uses:
 * h_out[g*F + f] = key(s_f . g), the OR of one table entry per key byte.
 * Checks the tables without a GPU. h_gens: k rows of n bytes, each a
 * permutation of 0..n-1. Returns CG_OK or CG_E_INVAL.
 */
int cg_test_host_expand_bits(int n, const uint8_t *h_gens, int k, const uint64_t *h_frontier,
                             uint64_t F, uint64_t *h_out);

#ifdef __cplusplus
}
#endif
#endif /* CAYLEYGROWTH_TESTING_H */
