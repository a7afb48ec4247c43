"""Each stage of the layer step on the GPU against a plain numpy reference
of the same operation, element by element (bit-exact: integer work)."""

import itertools
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2509_19162_amd import inputs as I  # noqa: E402
from paper_2509_19162_amd import testing as T  # noqa: E402


def np_pack(n, rows):
    rows = np.asarray(rows, dtype=np.uint64).reshape(-1, n)
    shifts = np.array([4 * (n - 1 - i) for i in range(n)], dtype=np.uint64)
    return np.bitwise_or.reduce(rows << shifts, axis=1) if n > 0 else np.zeros(len(rows), np.uint64)


def np_unpack(n, keys):
    keys = np.asarray(keys, dtype=np.uint64)
    return np.stack([(keys >> np.uint64(4 * (n - 1 - i))) & np.uint64(15) for i in range(n)], axis=1).astype(np.uint8)


def random_states(n, count, rng):
    return np.stack([rng.permutation(n) for _ in range(count)]).astype(np.uint8)


@pytest.fixture(scope="module")
def rng():
    return np.random.default_rng(19162)


@pytest.mark.parametrize("n", [2, 5, 8, 12, 16])
def test_pack_unpack_roundtrip(n, rng):
    rows = random_states(n, 3001, rng)
    keys = T.pack(n, rows)
    assert np.array_equal(T.to_u64(keys), np_pack(n, rows))
    assert np.array_equal(T.unpack(n, keys), rows)


@pytest.mark.parametrize("n", [2, 3, 7, 8, 9, 12, 15, 16])
@pytest.mark.parametrize("F", [1, 255, 4097, 70001])
def test_expand_matches_gather(n, F, rng):
    gens = [list(map(int, rng.permutation(n))) for _ in range(4)] + I.coxeter(n)[:2]
    rows = random_states(n, F, rng)
    frontier = T.from_u64(np_pack(n, rows))
    out = T.to_u64(T.expand(n, gens, frontier))
    expected = np.concatenate([np_pack(n, rows[:, g]) for g in gens])
    assert np.array_equal(out, expected)


def _stable_sorted(keys, lo, hi):
    mask = np.uint64((1 << (hi - lo)) - 1) if hi - lo < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    d = (keys >> np.uint64(lo)) & mask
    return keys[np.argsort(d, kind="stable")]


SORT_SIZES = [0, 1, 2, 3, 63, 64, 65, 4095, 4096, 4097, 8191, 8193, 100_003, 1_048_613]


@pytest.mark.parametrize("count", SORT_SIZES)
@pytest.mark.parametrize("lo,hi", [(4, 48), (0, 64), (4, 8), (12, 21)])
def test_sort_matches_stable_numpy(count, lo, hi, rng):
    keys = rng.integers(0, 2 ** 63, size=count, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, size=count, dtype=np.uint64)
    t = T.from_u64(keys)
    T.sort(t, lo, hi)
    assert np.array_equal(T.to_u64(t), _stable_sorted(keys, lo, hi))


@pytest.mark.parametrize("count", [5000, 300_000])
@pytest.mark.parametrize("distinct", [1, 3, 257])
def test_sort_heavy_duplicates(count, distinct, rng):
    pool = rng.integers(0, 2 ** 48, size=distinct, dtype=np.uint64)
    keys = pool[rng.integers(0, distinct, size=count)] | (rng.integers(0, 16, size=count, dtype=np.uint64))
    t = T.from_u64(keys)
    T.sort(t, 4, 48)
    assert np.array_equal(T.to_u64(t), _stable_sorted(keys, 4, 48))


# the 32-bit sort (ranks of candidates, n <= 12) has tiles of 15360 keys
SORT32_SIZES = [0, 1, 2, 65, 15359, 15360, 15361, 3 * 15360 + 7, 100_003, 1_048_613]


@pytest.mark.parametrize("count", SORT32_SIZES)
@pytest.mark.parametrize("lo,hi", [(0, 29), (0, 32), (3, 17), (8, 9)])
def test_sort32_matches_stable_numpy(count, lo, hi, rng):
    keys = rng.integers(0, 2 ** 32, size=count, dtype=np.uint64).astype(np.uint32)
    t = torch.from_numpy(keys.view(np.int32).copy()).cuda()
    T.sort32(t, lo, hi)
    got = t.cpu().numpy().view(np.uint32)
    digits = (keys.astype(np.uint64) >> np.uint64(lo)) & np.uint64((1 << (hi - lo)) - 1)
    assert np.array_equal(got, keys[np.argsort(digits, kind="stable")])


@pytest.mark.parametrize("count", [40_000, 2_000_000])
@pytest.mark.parametrize("distinct", [1, 5, 3000])
def test_sort32_duplicates_and_identity_passes(count, distinct, rng):
    # ranks below 2^20 sorted on 32 bits: the top pass is the identity (and
    # skipped for large arrays); many equal keys straddle tile borders
    pool = rng.integers(0, 1 << 20, size=distinct, dtype=np.uint64).astype(np.uint32)
    keys = pool[rng.integers(0, distinct, size=count)]
    t = torch.from_numpy(keys.view(np.int32).copy()).cuda()
    T.sort32(t, 0, 32)
    assert np.array_equal(t.cpu().numpy().view(np.uint32), np.sort(keys, kind="stable"))


@pytest.mark.parametrize("count,lo,hi", [(12_000_003, 4, 64), (9_437_185, 20, 60)])
def test_sort_large_persistent_blocks(count, lo, hi):
    # 64-bit passes run persistent blocks; past ~1500 resident blocks of
    # 4096-key tiles every block takes several tiles by ticket
    rng = np.random.default_rng(count)
    keys = rng.integers(0, 2 ** 63, size=count, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, size=count, dtype=np.uint64)
    t = T.from_u64(keys)
    T.sort(t, lo, hi)
    assert np.array_equal(T.to_u64(t), _stable_sorted(keys, lo, hi))


# Keys below 2^b sorted on all their bits in digits of balanced widths (the
# sort of 64-bit ranks and of binary states; 9 bits: two passes of 4 and 5).
SORT_BELOW_SIZES = [0, 1, 2, 65, 12287, 12288, 12289, 3 * 12288 + 5, 100_003, 1_048_613]


@pytest.mark.parametrize("count", SORT_BELOW_SIZES)
@pytest.mark.parametrize("bits", [8, 9, 17, 33, 38, 45, 48, 49, 64])
def test_sort_below_matches_numpy(count, bits, rng):
    if bits == 64:
        keys = rng.integers(0, 2 ** 63, size=count, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, size=count, dtype=np.uint64)
    else:
        keys = rng.integers(0, 2 ** bits, size=count, dtype=np.uint64)
    if count > 3:
        keys[:3] = [0, (1 << bits) - 1, (1 << bits) - 1]  # the extremes, one repeated
    t = T.from_u64(keys)
    T.sort_below(t, bits)
    assert np.array_equal(T.to_u64(t), np.sort(keys))


@pytest.mark.parametrize("count,bits", [(30_000_017, 45), (7_000_001, 38)])
def test_sort_below_large_persistent_blocks(count, bits):
    # 2441 and 570 tiles of 12288 keys against ~512 resident blocks: blocks
    # take several tiles each, and load the next one while writing one out
    rng = np.random.default_rng([count, bits])
    keys = rng.integers(0, 2 ** bits, size=count, dtype=np.uint64)
    keys[rng.integers(0, count, size=count // 3)] = keys[0]  # a heavy digit in every pass
    t = T.from_u64(keys)
    T.sort_below(t, bits)
    assert np.array_equal(T.to_u64(t), np.sort(keys))


def test_sort32_large():
    rng = np.random.default_rng(32)
    keys = rng.integers(0, 479001600, size=30_000_001, dtype=np.uint64).astype(np.uint32)
    t = torch.from_numpy(keys.view(np.int32).copy()).cuda()
    T.sort32(t, 0, 29)
    assert np.array_equal(t.cpu().numpy().view(np.uint32), np.sort(keys, kind="stable"))


def _np_dedup(s, a, b):
    u = np.unique(s)
    return np.setdiff1d(np.setdiff1d(u, a, assume_unique=True), b, assume_unique=True)


@pytest.mark.parametrize("C,na,nb", [(0, 0, 0), (1, 0, 0), (1, 1, 0), (4096, 100, 50),
                                     (4097, 5000, 5000), (100_000, 30_000, 10_000),
                                     (50_000, 400_000, 0), (200_000, 0, 150_000)])
def test_dedup_matches_numpy(C, na, nb, rng):
    universe = rng.integers(0, 2 ** 44, size=max(C // 3, 1), dtype=np.uint64) << np.uint64(4)
    s = np.sort(universe[rng.integers(0, len(universe), size=C)]) if C else np.zeros(0, np.uint64)
    a = np.unique(np.concatenate([rng.choice(universe, size=min(na, len(universe))),
                                  rng.integers(0, 2 ** 44, size=na, dtype=np.uint64) << np.uint64(4)]))[:na] if na else np.zeros(0, np.uint64)
    b = np.unique(np.concatenate([rng.choice(universe, size=min(nb, len(universe))),
                                  rng.integers(0, 2 ** 44, size=nb, dtype=np.uint64) << np.uint64(4)]))[:nb] if nb else np.zeros(0, np.uint64)
    out = T.dedup(T.from_u64(s), T.from_u64(a), T.from_u64(b))
    assert np.array_equal(T.to_u64(out), _np_dedup(s, a, b))


def test_layer_steps_reproduce_coxeter_layers():
    n = 7
    gens = I.coxeter(n)
    # reference layers by plain set arithmetic on numpy keys
    layers = [np_pack(n, np.arange(n, dtype=np.uint8)[None, :])]
    prev = np.zeros(0, np.uint64)
    while True:
        rows = np_unpack(n, layers[-1])
        cand = np.concatenate([np_pack(n, rows[:, g]) for g in gens])
        nxt = np.setdiff1d(np.setdiff1d(np.unique(cand), layers[-1]), prev)
        if len(nxt) == 0:
            break
        prev = layers[-1]
        layers.append(nxt)
    # the same walk through the GPU layer step
    f = T.from_u64(layers[0])
    p = T.from_u64(np.zeros(0, np.uint64))
    for d in range(1, len(layers)):
        out = T.layer_step(n, gens, f, p)
        assert np.array_equal(T.to_u64(out), layers[d]), d
        p, f = f, out
    assert T.layer_step(n, gens, f, p).numel() == 0


@pytest.mark.parametrize("nbytes", [16, 4096 + 16 * 7, 1 << 22])
def test_copy_kernel_copies(nbytes, rng):
    src = torch.from_numpy(rng.integers(0, 256, nbytes, dtype=np.uint8)).cuda()
    dst = torch.zeros_like(src)
    T.copy(src, dst, repeats=2)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


@pytest.fixture
def rts_min():
    old = os.environ.get("CG_SORT_RTS_MIN")

    def set_(v):
        os.environ["CG_SORT_RTS_MIN"] = str(v)

    yield set_
    if old is None:
        os.environ.pop("CG_SORT_RTS_MIN", None)
    else:
        os.environ["CG_SORT_RTS_MIN"] = old


@pytest.mark.parametrize("mode", ["reduce_then_scan", "lookback"])
@pytest.mark.parametrize("count,lo,hi", [(1, 0, 64), (4097, 4, 48), (8193 * 3 + 5, 0, 64), (300001, 4, 44),
                                         ((1 << 20) + 37, 8, 40)])
def test_sort_both_pass_modes(mode, count, lo, hi, rng, rts_min):
    rts_min(1 if mode == "reduce_then_scan" else 0)
    keys = rng.integers(0, 1 << 63, size=count, dtype=np.int64).astype(np.uint64)
    keys[: count // 3] = keys[0]  # a heavy repeat
    d = T.from_u64(keys)
    T.sort(d, lo, hi)
    got = T.to_u64(d)
    field = (keys >> np.uint64(lo)) & np.uint64((1 << (hi - lo)) - 1) if hi - lo < 64 else keys
    exp = keys[np.argsort(field, kind="stable")]
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("fam,n", [("pancake", 9), ("lrx", 10), ("all_transpositions", 8)])
def test_growth_with_reduce_then_scan(fam, n, rts_min, oracle_c):
    from paper_2509_19162_amd import api

    rts_min(1)
    gens = I.family(fam, n)
    exp = oracle_c.growth(n, gens, max_layers=512)[0]
    assert api.growth_ex(n, gens, max_layers=512).sizes == exp
    assert api.growth_ex(n, gens, max_layers=512, packed_sort=True).sizes == exp
