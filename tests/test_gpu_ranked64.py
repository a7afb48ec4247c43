"""Growth of S_13..S_16 with candidates sorted and deduplicated as 64-bit
lexicographic ranks (the default for a permutation start from n = 13)
against the oracle and against the packed-key sort path. Runs stop at the
first layer above a frontier limit so the oracle finishes in seconds, and
every family, start, stop rule, layer export and chunked layer is compared
layer by layer. Tolerance: none (exact integers)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2509_19162_amd import _native as N  # noqa: E402
from paper_2509_19162_amd import api  # noqa: E402
from paper_2509_19162_amd import inputs as I  # noqa: E402

LIMIT = 150_000


def _check(n, gens, oracle_c, start=None, directed=False, limit=LIMIT, max_layers=512):
    r = api.growth_ex(n, gens, max_layers=max_layers, max_frontier=limit, start=start, allow_directed=directed)
    p = api.growth_ex(n, gens, max_layers=max_layers, max_frontier=limit, start=start, allow_directed=directed,
                      packed_sort=True)
    exp, rc, _ = oracle_c.growth(n, gens, max_layers=max_layers, max_frontier=limit, start=start)
    assert r.sizes == exp and r.status == rc, (n, r.sizes[:8], exp[:8])
    assert p.sizes == exp and p.status == rc
    assert r.states_expanded == (sum(exp[:-1]) if rc == 1 else sum(exp))
    return r


@pytest.mark.parametrize("n", [13, 14, 15, 16])
@pytest.mark.parametrize("fam", ["lrx", "pancake", "coxeter", "star", "reversals"])
def test_families_match_oracle(n, fam, oracle_c):
    _check(n, I.family(fam, n), oracle_c)


@pytest.mark.parametrize("n", [13, 16])
def test_all_transpositions_match_stirling_prefix(n, oracle_c):
    _check(n, I.all_transpositions(n), oracle_c, limit=20_000)


@pytest.mark.parametrize("n", [13, 14, 15, 16])
@pytest.mark.parametrize("seed", [0, 1])
def test_random_sets_and_starts(n, seed, oracle_c):
    rng = np.random.default_rng([I.SEED, n, seed])
    gens = I.random_perms_with_inverses(n, int(rng.integers(1, 4)), rng)
    start = [int(x) for x in rng.permutation(n)]
    _check(n, gens, oracle_c)
    _check(n, gens, oracle_c, start=start)


@pytest.mark.parametrize("n", [13, 16])
def test_directed_lx(n, oracle_c):
    _check(n, I.lx(n), oracle_c, directed=True, limit=50_000)


def test_stop_rule_max_layers(oracle_c):
    r = _check(16, I.lrx(16), oracle_c, max_layers=12)
    assert r.status == N.CG_TRUNCATED and len(r.sizes) == 12


def test_layer_contents_match_oracle(oracle_c):
    n = 14
    gens = I.pancake(n)
    r = api.growth_ex(n, gens, max_layers=5, export_layers=200_000)
    sizes, rc, states = oracle_c.growth(n, gens, max_layers=5, with_states=True)
    assert r.sizes == sizes
    off = 0
    for d, sz in enumerate(sizes):
        got = np.asarray(r.layers[d])
        exp = np.unique(np.asarray(states[off: off + sz], dtype=np.uint8).reshape(-1, n), axis=0)
        off += sz
        # each layer comes out in increasing lexicographic order
        assert np.array_equal(got, exp), d


def test_chunked_layers_and_keep_all(oracle_c, monkeypatch):
    n = 16
    gens = I.lrx(16)
    exp, rc, _ = oracle_c.growth(n, gens, max_layers=512, max_frontier=400_000)
    monkeypatch.setenv("CG_CHUNK_CANDIDATES", "100000")
    r = api.growth_ex(n, gens, max_layers=512, max_frontier=400_000)
    assert r.sizes == exp and r.status == rc
    monkeypatch.delenv("CG_CHUNK_CANDIDATES")
    k = api.growth_ex(n, gens, max_layers=512, max_frontier=400_000, keep_all_layers=True)
    assert k.sizes == exp and k.status == rc


@pytest.mark.parametrize("n", [13, 14, 15, 16])
def test_rank64_on_device_matches_host(n):
    rng = np.random.default_rng(n)
    rows = np.stack([rng.permutation(n) for _ in range(20000)]).astype(np.uint64)
    keys = np.ascontiguousarray(np.bitwise_or.reduce(
        rows << np.array([4 * (n - 1 - i) for i in range(n)], dtype=np.uint64), axis=1))
    dev = np.zeros(len(keys), dtype=np.uint64)
    host = np.zeros(len(keys), dtype=np.uint64)
    lib = N.lib()
    assert lib.cg_test_rank64(n, keys.ctypes.data_as(N.u64p), len(keys), dev.ctypes.data_as(N.u64p), 1, None) == 0
    assert lib.cg_test_rank64(n, keys.ctypes.data_as(N.u64p), len(keys), host.ctypes.data_as(N.u64p), 0, None) == 0
    assert np.array_equal(dev, host)
    back = np.zeros(len(keys), dtype=np.uint64)
    assert lib.cg_test_unrank64(n, dev.ctypes.data_as(N.u64p), len(keys), back.ctypes.data_as(N.u64p), 1,
                                None) == 0
    assert np.array_equal(back, keys)
