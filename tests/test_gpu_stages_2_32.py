"""Sort and dedup stages beyond 2^32 keys, checked element by element.

The S_16 LRX growth to 2^31 is the one workload whose expansions pass 2^32
candidates, so the 64-bit digit offsets, look-back values, tile counts and
output offsets of these stages carry values above 2^32 only there. These
tests drive the same kernels through the testing ABI with inputs whose
sorted or deduplicated output is known in closed form:
  * sort: the keys are a bijective scramble i -> (a*i + b) mod N of
    0..N-1 (a prime, coprime to N), so the stable sorted output is
    0, 1, ..., N-1;
  * 32-bit sort: the same scramble cut to its low 32 bits, so every value
    below N - 2^32 appears twice and every other value once;
  * dedup: each value v < U twice, with the multiples of 3 in one reference
    layer and the multiples of 5 that are not multiples of 3 in the other,
    so the survivors are the v < U prime to 15, eight in every fifteen.
Inputs are generated on the device and checked in slices of 2^28 elements:
no single torch operation touches more than 2^32 elements (on this ROCm
build, elementwise torch operations over one tensor of more than 2^32
elements gave wrong values).
Tolerance: none.
"""

import ctypes

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2509_19162_amd import _native as N  # noqa: E402
from paper_2509_19162_amd import testing as T  # noqa: E402

DELTA = 4097
N_KEYS = (1 << 32) + DELTA
A = 1_000_000_007  # prime, and N_KEYS is not a multiple of it
B = 123_456_789
SLICE = 1 << 28


@pytest.fixture(autouse=True)
def _fresh_memory():
    torch.cuda.synchronize()
    N.lib().cg_release_cached_memory()
    torch.cuda.empty_cache()
    yield
    torch.cuda.synchronize()
    N.lib().cg_release_cached_memory()
    torch.cuda.empty_cache()


def _scramble(n, dtype=torch.int64):
    """(A*i + B) mod n for i = 0..n-1 (a bijection), cut to `dtype`."""
    assert n % A != 0
    x = torch.empty(n, dtype=dtype, device="cuda")
    for s in range(0, n, SLICE):
        e = min(n, s + SLICE)
        v = torch.arange(s, e, dtype=torch.int64, device="cuda")
        v.mul_(A).add_(B).remainder_(n)  # A*i + B < 2^63 for n < 2^33
        x[s:e] = v.to(dtype)  # int32: the low 32 bits
    return x


def test_sort64_beyond_2_32_keys():
    print("64-bit sort of", N_KEYS, "scrambled keys", flush=True)
    keys = _scramble(N_KEYS)
    tmp = torch.empty_like(keys)
    rc = N.lib().cg_test_sort(T._dptr(keys), T._dptr(tmp), N_KEYS, 0, 33, T._stream(None))
    assert rc == N.CG_OK, N.lib().cg_last_error()
    del tmp
    N.lib().cg_release_cached_memory()
    torch.cuda.synchronize()
    for s in range(0, N_KEYS, SLICE):
        e = min(N_KEYS, s + SLICE)
        exp = torch.arange(s, e, dtype=torch.int64, device="cuda")
        assert torch.equal(keys[s:e], exp), s


def test_sort64_balanced_digits_beyond_2_32_keys():
    """The same keys sorted on bits [0, 33) in balanced digits (6,6,7,7,7),
    as the sorts of 64-bit ranks and binary states run."""
    print("64-bit sort in balanced digits of", N_KEYS, "scrambled keys", flush=True)
    keys = _scramble(N_KEYS)
    tmp = torch.empty_like(keys)
    rc = N.lib().cg_test_sort_below(T._dptr(keys), T._dptr(tmp), N_KEYS, 33, T._stream(None))
    assert rc == N.CG_OK, N.lib().cg_last_error()
    del tmp
    N.lib().cg_release_cached_memory()
    torch.cuda.synchronize()
    for s in range(0, N_KEYS, SLICE):
        e = min(N_KEYS, s + SLICE)
        exp = torch.arange(s, e, dtype=torch.int64, device="cuda")
        assert torch.equal(keys[s:e], exp), s


def test_sort32_beyond_2_32_keys():
    print("32-bit sort of", N_KEYS, "keys with", DELTA, "repeated values", flush=True)
    keys = _scramble(N_KEYS, torch.int32)
    tmp = torch.empty_like(keys)
    rc = N.lib().cg_test_sort32(T._dptr(keys), T._dptr(tmp), N_KEYS, 0, 32, T._stream(None))
    assert rc == N.CG_OK, N.lib().cg_last_error()
    del tmp
    N.lib().cg_release_cached_memory()
    torch.cuda.synchronize()
    # values 0..DELTA-1 twice, then DELTA..2^32-1 once (as 32-bit patterns)
    head = torch.arange(DELTA, dtype=torch.int64, device="cuda").repeat_interleave(2).to(torch.int32)
    assert torch.equal(keys[: 2 * DELTA], head)
    for s in range(2 * DELTA, N_KEYS, SLICE):
        e = min(N_KEYS, s + SLICE)
        exp = torch.arange(s - DELTA, e - DELTA, dtype=torch.int64, device="cuda").to(torch.int32)
        assert torch.equal(keys[s:e], exp), s


def test_dedup_beyond_2_32_candidates():
    U = (1 << 31) + DELTA  # distinct values
    C = 2 * U  # > 2^32 candidates, each value twice
    print("dedup of", C, "candidates against two reference layers", flush=True)
    cand = torch.empty(C, dtype=torch.int64, device="cuda")
    for s in range(0, C, SLICE):
        e = min(C, s + SLICE)
        cand[s:e] = torch.arange(s, e, dtype=torch.int64, device="cuda").bitwise_right_shift_(1)
    a = torch.arange(0, U, 3, dtype=torch.int64, device="cuda")
    v5 = torch.arange(0, U, 5, dtype=torch.int64, device="cuda")
    b = v5[v5.remainder(3) != 0].contiguous()
    del v5
    out = torch.empty(C, dtype=torch.int64, device="cuda")
    cnt = ctypes.c_uint64(0)
    rc = N.lib().cg_test_dedup(T._dptr(cand), C, T._dptr(a), a.numel(), T._dptr(b), b.numel(), T._dptr(out),
                               ctypes.byref(cnt), T._stream(None))
    assert rc == N.CG_OK, N.lib().cg_last_error()
    del cand, a, b
    N.lib().cg_release_cached_memory()
    torch.cuda.empty_cache()
    pat = torch.tensor([1, 2, 4, 7, 8, 11, 13, 14], dtype=torch.int64, device="cuda")
    full, rem = divmod(U, 15)
    expected = 8 * full + int((pat < rem).sum())
    assert cnt.value == expected
    for s in range(0, expected, SLICE):
        e = min(expected, s + SLICE)
        i = torch.arange(s, e, dtype=torch.int64, device="cuda")
        exp = 15 * (i // 8) + pat[i % 8]
        assert torch.equal(out[s:e], exp), s
