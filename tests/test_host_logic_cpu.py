"""Host-side logic of the library checked on the CPU (no device calls):
lexicographic rank/unrank of packed keys and the byte-permute selector
tables of the expand step (v_perm_b32 semantics emulated on the host)."""

import ctypes
import itertools
import math

import numpy as np
import pytest

from paper_2509_19162_amd import _native as N
from paper_2509_19162_amd import inputs as I


def pack(n, rows):
    rows = np.asarray(rows, dtype=np.uint64).reshape(-1, n)
    shifts = np.array([4 * (n - 1 - i) for i in range(n)], dtype=np.uint64)
    return np.bitwise_or.reduce(rows << shifts, axis=1)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 9])
def test_rank_is_lexicographic_index(n):
    perms = list(itertools.permutations(range(n)))  # lexicographic order
    keys = np.ascontiguousarray(pack(n, perms))
    ranks = np.zeros(len(perms), dtype=np.uint32)
    rc = N.lib().cg_test_rank(n, keys.ctypes.data_as(N.u64p), len(perms),
                              ranks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), 0, None)
    assert rc == 0
    assert np.array_equal(ranks, np.arange(len(perms), dtype=np.uint32))
    back = np.zeros(len(perms), dtype=np.uint64)
    rc = N.lib().cg_test_unrank(n, ranks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), len(perms),
                                back.ctypes.data_as(N.u64p), 0, None)
    assert rc == 0 and np.array_equal(back, keys)


@pytest.mark.parametrize("n", [10, 11, 12])
def test_rank_sampled_large_n(n):
    rng = np.random.default_rng(n)
    perms = [list(map(int, rng.permutation(n))) for _ in range(500)]
    keys = np.ascontiguousarray(pack(n, perms))
    ranks = np.zeros(len(perms), dtype=np.uint32)
    N.lib().cg_test_rank(n, keys.ctypes.data_as(N.u64p), len(perms),
                         ranks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), 0, None)
    # Lehmer code by its definition, in Python integers
    for p, r in zip(perms, ranks):
        code = sum(sum(1 for j in range(i + 1, n) if p[j] < p[i]) * math.factorial(n - 1 - i) for i in range(n))
        assert code == int(r)
    order = np.argsort(keys, kind="stable")
    assert np.all(np.diff(ranks[order].astype(np.int64)) > 0)  # order preserved
    # unrank inverts it; rank 0 is the identity and n! - 1 the reversal
    rs = np.ascontiguousarray(np.concatenate([ranks, [0, math.factorial(n) - 1]]).astype(np.uint32))
    back = np.zeros(len(rs), dtype=np.uint64)
    assert N.lib().cg_test_unrank(n, rs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), len(rs),
                                  back.ctypes.data_as(N.u64p), 0, None) == 0
    assert np.array_equal(back[:-2], keys)
    assert int(back[-2]) == int(pack(n, [list(range(n))])[0])
    assert int(back[-1]) == int(pack(n, [list(range(n))[::-1]])[0])


def test_rank_rejects_bad_input():
    r = np.zeros(1, dtype=np.uint32)
    k = np.zeros(1, dtype=np.uint64)
    assert N.lib().cg_test_rank(13, k.ctypes.data_as(N.u64p), 1,
                                r.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), 0, None) == N.CG_E_INVAL
    r[0] = 6
    assert N.lib().cg_test_unrank(3, r.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), 1,
                                  k.ctypes.data_as(N.u64p), 0, None) == N.CG_E_INVAL


@pytest.mark.parametrize("n", [1, 2, 3, 8, 9, 12, 15, 16])
def test_host_expand_selectors_match_gather(n):
    rng = np.random.default_rng(100 + n)
    gens = [list(map(int, rng.permutation(n))) for _ in range(5)] + I.coxeter(n)[:2]
    rows = np.stack([rng.permutation(n) for _ in range(200)]).astype(np.uint8)
    keys = np.ascontiguousarray(pack(n, rows))
    g = np.ascontiguousarray(np.asarray(gens, dtype=np.uint8))
    out = np.zeros(len(gens) * len(keys), dtype=np.uint64)
    rc = N.lib().cg_test_host_expand(n, g.ctypes.data_as(N.u8p), len(gens), keys.ctypes.data_as(N.u64p),
                                     len(keys), out.ctypes.data_as(N.u64p))
    assert rc == 0
    expected = np.concatenate([pack(n, rows[:, gg]) for gg in gens])
    assert np.array_equal(out, expected)


def _lehmer_rank(p):
    """The lexicographic index by its definition (Lehmer code), in Python
    integers."""
    n = len(p)
    return sum(sum(1 for j in range(i + 1, n) if p[j] < p[i]) * math.factorial(n - 1 - i) for i in range(n))


@pytest.mark.parametrize("n", [13, 14, 15, 16])
def test_rank64_sampled(n):
    """64-bit ranks (n = 13..16) against the Lehmer code written out, with
    the order preserved and unrank inverting them; rank 0 is the identity,
    n! - 1 the reversal, and the neighbours of both ends of every split of
    the Horner sum round-trip too."""
    rng = np.random.default_rng(1000 + n)
    perms = [list(map(int, rng.permutation(n))) for _ in range(400)]
    perms += [list(range(n)), list(range(n))[::-1]]
    keys = np.ascontiguousarray(pack(n, perms))
    ranks = np.zeros(len(perms), dtype=np.uint64)
    assert N.lib().cg_test_rank64(n, keys.ctypes.data_as(N.u64p), len(perms), ranks.ctypes.data_as(N.u64p),
                                  0, None) == 0
    for p, r in zip(perms, ranks):
        assert _lehmer_rank(p) == int(r)
    assert int(ranks[-2]) == 0 and int(ranks[-1]) == math.factorial(n) - 1
    order = np.argsort(keys, kind="stable")
    assert np.all(np.diff(ranks[order].astype(object)) > 0)
    # ranks around multiples of the low radices (carries between the parts)
    extra = []
    for m in (720, 40320, 362880, 3628800, 479001600):
        for q in (1, 7, 12345):
            v = q * m
            extra += [v - 1, v, v + 1]
    extra = [v for v in extra if 0 <= v < math.factorial(n)]
    rs = np.ascontiguousarray(np.concatenate([ranks, np.asarray(extra, dtype=np.uint64)]).astype(np.uint64))
    back = np.zeros(len(rs), dtype=np.uint64)
    assert N.lib().cg_test_unrank64(n, rs.ctypes.data_as(N.u64p), len(rs), back.ctypes.data_as(N.u64p), 0,
                                    None) == 0
    assert np.array_equal(back[: len(keys)], keys)
    again = np.zeros(len(rs), dtype=np.uint64)
    assert N.lib().cg_test_rank64(n, back.ctypes.data_as(N.u64p), len(rs), again.ctypes.data_as(N.u64p), 0,
                                  None) == 0
    assert np.array_equal(again, rs)
    for v, k in zip(extra, back[len(keys):]):
        row = [(int(k) >> (4 * (n - 1 - i))) & 15 for i in range(n)]
        assert sorted(row) == list(range(n)) and _lehmer_rank(row) == v


@pytest.mark.parametrize("n", [13, 14, 15, 16])
def test_unrank64_many_ranks_round_trip(n):
    """200,000 random ranks below n!: unrank gives a permutation (n distinct
    nibbles) whose rank (checked against the Lehmer code above) is the rank
    it came from, so every digit of the split division chain is exact."""
    rng = np.random.default_rng(2000 + n)
    rs = np.ascontiguousarray(rng.integers(0, math.factorial(n), size=200_000, dtype=np.uint64))
    keys = np.zeros(len(rs), dtype=np.uint64)
    assert N.lib().cg_test_unrank64(n, rs.ctypes.data_as(N.u64p), len(rs), keys.ctypes.data_as(N.u64p), 0,
                                    None) == 0
    nib = np.stack([(keys >> np.uint64(4 * (n - 1 - i))) & np.uint64(15) for i in range(n)], axis=1)
    assert np.array_equal(np.sort(nib, axis=1), np.broadcast_to(np.arange(n, dtype=np.uint64), nib.shape))
    back = np.zeros(len(rs), dtype=np.uint64)
    assert N.lib().cg_test_rank64(n, keys.ctypes.data_as(N.u64p), len(rs), back.ctypes.data_as(N.u64p), 0,
                                  None) == 0
    assert np.array_equal(back, rs)


def test_rank64_rejects_bad_input():
    r = np.zeros(1, dtype=np.uint64)
    k = np.zeros(1, dtype=np.uint64)
    assert N.lib().cg_test_rank64(12, k.ctypes.data_as(N.u64p), 1, r.ctypes.data_as(N.u64p), 0, None) == N.CG_E_INVAL
    r[0] = math.factorial(13)
    assert N.lib().cg_test_unrank64(13, r.ctypes.data_as(N.u64p), 1, k.ctypes.data_as(N.u64p), 0,
                                    None) == N.CG_E_INVAL


def pack_bits(n, rows):
    rows = np.asarray(rows, dtype=np.uint64).reshape(-1, n)
    shifts = np.array([n - 1 - i for i in range(n)], dtype=np.uint64)
    return np.bitwise_or.reduce(rows << shifts, axis=1)


@pytest.mark.parametrize("n", [1, 2, 7, 8, 9, 17, 24, 31, 32, 33, 40, 57, 63, 64])
def test_host_expand_bits_matches_gather(n):
    """Binary states (one bit per entry): the byte tables of the bit
    permutation, applied on the host, give key(s . g) with t[i] = s[g[i]]
    for random 0/1 vectors and random permutations."""
    rng = np.random.default_rng(500 + n)
    gens = [list(map(int, rng.permutation(n))) for _ in range(6)]
    if n > 1:
        gens.append([n - 1 - i for i in range(n)])  # the full reversal
        gens.append([(i + 1) % n for i in range(n)])  # a rotation
    rows = rng.integers(0, 2, size=(300, n)).astype(np.uint8)
    rows[0] = 0
    rows[1] = 1
    keys = np.ascontiguousarray(pack_bits(n, rows))
    g = np.ascontiguousarray(np.asarray(gens, dtype=np.uint8))
    out = np.zeros(len(gens) * len(keys), dtype=np.uint64)
    rc = N.lib().cg_test_host_expand_bits(n, g.ctypes.data_as(N.u8p), len(gens), keys.ctypes.data_as(N.u64p),
                                          len(keys), out.ctypes.data_as(N.u64p))
    assert rc == 0
    expected = np.concatenate([pack_bits(n, rows[:, gg]) for gg in gens])
    assert np.array_equal(out, expected)


def test_host_expand_bits_rejects_bad_rows():
    k = np.zeros(1, dtype=np.uint64)
    o = np.zeros(1, dtype=np.uint64)
    bad = np.zeros((1, 20), dtype=np.uint8)  # not a permutation
    assert N.lib().cg_test_host_expand_bits(20, bad.ctypes.data_as(N.u8p), 1, k.ctypes.data_as(N.u64p), 1,
                                            o.ctypes.data_as(N.u64p)) == N.CG_E_INVAL
    g = np.arange(65, dtype=np.uint8).reshape(1, 65)
    assert N.lib().cg_test_host_expand_bits(65, g.ctypes.data_as(N.u8p), 1, k.ctypes.data_as(N.u64p), 1,
                                            o.ctypes.data_as(N.u64p)) == N.CG_E_INVAL
