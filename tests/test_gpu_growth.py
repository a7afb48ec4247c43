"""Growth on the GPU (through the C ABI) against the CPU oracle, closed
forms and the paper's printed values. Tolerance: none (exact integers)."""

import json
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from golden_data import GOLDEN, binary_coset_growth, mahonian, max_diameter_table, transposition_growth  # noqa: E402
from oracle import bfs_set  # noqa: E402
from paper_2509_19162_amd import _native as N  # noqa: E402
from paper_2509_19162_amd import api  # noqa: E402
from paper_2509_19162_amd import inputs as I  # noqa: E402

FAMS = ["coxeter", "cyclic_coxeter", "all_transpositions", "star", "pancake", "lrx", "reversals",
        "transposons", "three_cycles"]


def test_bubble_sort_graph_s8():
    """S_8 with the 7 adjacent transpositions: Mahonian layers, diameter 28."""
    sizes = api.growth(8, I.coxeter(8))
    assert sizes == mahonian(8)
    assert len(sizes) - 1 == 28 and sum(sizes) == 40320


@pytest.mark.parametrize("fam", FAMS)
@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7, 8, 9])
def test_families_match_oracle(fam, n, oracle_c):
    gens = I.family(fam, n)
    if not gens:
        pytest.skip("empty family")
    expected, rc, _ = oracle_c.growth(n, gens)
    r = api.growth_ex(n, gens)
    assert r.sizes == expected and r.status == rc == 0


@pytest.mark.parametrize("full", [False, True], ids=["incremental", "full"])
@pytest.mark.parametrize("fam,n", [("pancake", 8), ("coxeter", 9), ("star", 7), ("lrx", 8), ("all_transpositions", 7),
                                   ("three_cycles", 6)])
def test_incremental_and_full_ranks(fam, n, full, oracle_c, monkeypatch):
    # candidates' ranks reuse the parent's Lehmer digits past each
    # generator's last moved position, or (CG_RANK_FULL) are computed whole
    if full:
        monkeypatch.setenv("CG_RANK_FULL", "1")
    gens = I.family(fam, n)
    expected, rc, _ = oracle_c.growth(n, gens)
    r = api.growth_ex(n, gens, keep_all_layers=True, export_layers=math.factorial(n))
    assert r.sizes == expected and r.status == rc == 0
    if full:
        monkeypatch.delenv("CG_RANK_FULL")
        other = api.growth_ex(n, gens, keep_all_layers=True, export_layers=math.factorial(n))
        assert other.sizes == r.sizes
        for a, b in zip(other.layers, r.layers):
            assert np.array_equal(np.asarray(a), np.asarray(b))


@pytest.mark.parametrize("n", [10, 11, 12])
def test_closed_forms_beyond_the_python_oracle(n):
    assert api.growth(n, I.coxeter(n), max_layers=100) == mahonian(n)
    if n <= 11:
        assert api.growth(n, I.all_transpositions(n)) == transposition_growth(n)


@pytest.mark.parametrize("seed", range(12))
def test_random_sets_match_oracle(seed, oracle_c):
    rng = I.rng_for(seed, seed=7)
    n = int(rng.integers(5, 10))
    gens = I.random_perms_with_inverses(n, int(rng.integers(1, 4)), rng)
    expected, _, _ = oracle_c.growth(n, gens)
    assert api.growth(n, gens, max_layers=4096) == expected


@pytest.mark.parametrize("seed", range(4))
def test_layer_contents_match_oracle(seed):
    rng = I.rng_for(100 + seed, seed=7)
    n = 6 + seed % 3
    gens = I.random_involutions(n, 3, rng)
    layers, complete = bfs_set.bfs_layers(n, gens)
    total = sum(len(x) for x in layers)
    r = api.growth_ex(n, gens, export_layers=total)
    assert complete and r.status == N.CG_OK
    assert r.sizes == [len(x) for x in layers]
    for got, exp in zip(r.layers, layers):
        exp_sorted = np.array(sorted(exp), dtype=np.uint8)
        assert np.array_equal(got, exp_sorted)


@pytest.mark.parametrize("row", max_diameter_table(directed=False), ids=lambda r: f"n{r[0]}")
def test_paper_max_diameters(row):
    n, diam, gens = row
    if n > 14:
        pytest.skip("S_15 does not fit one device in any engine")
    # S_13 and S_14 (14! = 8.7e10 states) run in the bitmask engine
    r = api.growth_ex(n, gens, max_layers=512, bitmask=n >= 13)
    assert r.status == N.CG_OK
    assert len(r.sizes) - 1 == diam
    assert sum(r.sizes) == math.factorial(n)


@pytest.mark.parametrize("seed", range(4))
def test_metamorphic_invariance(seed, oracle_c):
    rng = I.rng_for(200 + seed, seed=7)
    n = int(rng.integers(7, 11))
    gens = I.random_perms_with_inverses(n, 2, rng)
    base = api.growth_ex(n, gens, max_layers=4096)
    start = [int(x) for x in rng.permutation(n)]
    assert api.growth_ex(n, gens, max_layers=4096, start=start).sizes == base.sizes
    h = [int(x) for x in rng.permutation(n)]
    conj = [I.compose(I.compose(I.inverse(h), g), h) for g in gens]
    assert api.growth_ex(n, conj, max_layers=4096).sizes == base.sizes
    shuffled = [gens[i] for i in rng.permutation(len(gens))] + gens[:2] + [list(range(n))]
    assert api.growth_ex(n, shuffled, max_layers=4096).sizes == base.sizes
    assert api.growth_ex(n, gens, max_layers=4096, keep_all_layers=True).sizes == base.sizes


def test_stop_rules_match_oracle(oracle_c):
    gens = I.lrx(10)
    for ml in (1, 2, 7, 20):
        exp, rc, _ = oracle_c.growth(10, gens, max_layers=ml)
        r = api.growth_ex(10, gens, max_layers=ml)
        assert r.sizes == exp and r.status == rc
    for mf in (1, 100, 5000):
        exp, rc, _ = oracle_c.growth(10, gens, max_frontier=mf)
        r = api.growth_ex(10, gens, max_frontier=mf, max_layers=4096)
        assert r.sizes == exp and r.status == rc == N.CG_TRUNCATED


def test_degenerate_inputs():
    assert api.growth(1, [[0]]) == [1]
    assert api.growth(4, [[0, 1, 2, 3]]) == [1]
    assert api.growth(2, [[1, 0]]) == [1, 1]
    r = api.growth_ex(5, I.coxeter(5), max_layers=1)
    assert r.sizes == [1] and r.status == N.CG_TRUNCATED


@pytest.mark.parametrize("fam", ["reversals", "transposons"])
@pytest.mark.parametrize("n", [6, 9, 12, 16])
def test_binary_coset_start(fam, n, oracle_c):
    start = I.binary_central_state(n)
    gens = I.family(fam, n)
    r = api.growth_ex(n, gens, start=start, max_layers=64)
    if n <= 12:
        exp, rc, _ = oracle_c.growth(n, gens, start=start)
        assert r.sizes == exp
    assert r.sizes == binary_coset_growth(n)


def _stored(name):
    path = os.path.join(GOLDEN, "oracle_growth.json")
    if not os.path.exists(path):
        pytest.skip("oracle fixtures not generated")
    with open(path) as f:
        d = json.load(f)
    if name not in d:
        pytest.skip(f"{name} not in oracle fixtures")
    return d[name]


def test_pancake_s12_full_growth_matches_oracle():
    """S_12 with the 11 prefix reversals, every layer kept on the device."""
    exp = _stored("pancake_12")
    r = api.growth_ex(12, I.pancake(12), keep_all_layers=True)
    assert r.status == N.CG_OK
    assert r.sizes == exp["sizes"]
    assert sum(r.sizes) == math.factorial(12)


def test_pancake_s12_full_run_first_layers_match_oracle(oracle_c):
    """The full S_12 growth (all layers kept, as benchmarked) exports its
    first states; layers 0..6 (622,438 states) must equal the oracle's."""
    r = api.growth_ex(12, I.pancake(12), keep_all_layers=True, export_layers=700_000)
    assert r.status == N.CG_OK and sum(r.sizes) == math.factorial(12)
    sizes, rc, states = oracle_c.growth(12, I.pancake(12), max_layers=7, with_states=True)
    assert r.sizes[:7] == sizes
    off = 0
    for d, sz in enumerate(sizes):
        got = np.asarray(r.layers[d])
        exp = states[off: off + sz]
        off += sz
        key = lambda a: np.unique(np.asarray(a, dtype=np.uint8).reshape(-1, 12), axis=0)
        assert np.array_equal(key(got), key(exp)), d


@pytest.mark.parametrize("n", [2, 7, 12])
def test_rank_on_device_matches_host(n):
    import ctypes

    rng = np.random.default_rng(n)
    rows = np.stack([rng.permutation(n) for _ in range(5000)]).astype(np.uint64)
    keys = np.ascontiguousarray(np.bitwise_or.reduce(rows << np.array([4 * (n - 1 - i) for i in range(n)], dtype=np.uint64), axis=1))
    u32p = ctypes.POINTER(ctypes.c_uint32)
    dev = np.zeros(len(keys), dtype=np.uint32)
    host = np.zeros(len(keys), dtype=np.uint32)
    assert N.lib().cg_test_rank(n, keys.ctypes.data_as(N.u64p), len(keys), dev.ctypes.data_as(u32p), 1, None) == 0
    assert N.lib().cg_test_rank(n, keys.ctypes.data_as(N.u64p), len(keys), host.ctypes.data_as(u32p), 0, None) == 0
    assert np.array_equal(dev, host)
    back = np.zeros(len(keys), dtype=np.uint64)
    assert N.lib().cg_test_unrank(n, dev.ctypes.data_as(u32p), len(keys), back.ctypes.data_as(N.u64p), 1, None) == 0
    assert np.array_equal(back, keys)


@pytest.mark.parametrize("fam", ["pancake", "all_transpositions", "lrx", "reversals"])
@pytest.mark.parametrize("n", [5, 9, 11])
def test_ranked_and_packed_sorts_agree(fam, n, oracle_c):
    gens = I.family(fam, n)
    a = api.growth_ex(n, gens, max_layers=256)
    b = api.growth_ex(n, gens, max_layers=256, packed_sort=True)
    assert a.sizes == b.sizes
    if n <= 9:
        assert a.sizes == oracle_c.growth(n, gens)[0]
    elif fam == "all_transpositions":
        assert a.sizes == transposition_growth(n)  # Stirling numbers of the first kind
    else:
        assert a.sizes == _stored(f"family_{n}")[fam]["sizes"]
    # same layer contents on a small case
    if n == 5:
        ea = api.growth_ex(n, gens, export_layers=120)
        eb = api.growth_ex(n, gens, export_layers=120, packed_sort=True)
        for x, y in zip(ea.layers, eb.layers):
            assert np.array_equal(x, y)


def test_growth_from_several_host_threads(oracle_c):
    """cg_growth from eight host threads at once (each call runs on a stream
    of its own), three calls each, every result checked against the
    oracle."""
    import threading

    jobs = [(n, I.family(fam, n)) for n, fam in
            [(8, "coxeter"), (9, "pancake"), (7, "all_transpositions"), (9, "lrx"), (8, "star"),
             (9, "reversals"), (6, "coxeter"), (9, "star")]]
    got = [[] for _ in jobs]
    errors = []

    def work(i):
        try:
            for _ in range(3):
                got[i].append(api.growth(*jobs[i], max_layers=256))
        except Exception as e:  # surfaced below
            errors.append(e)

    th = [threading.Thread(target=work, args=(i,)) for i in range(len(jobs))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    for (n, g), runs in zip(jobs, got):
        exp = oracle_c.growth(n, g)[0]
        assert runs == [exp] * 3, n


def test_memory_stats_track_the_buffers_of_a_run():
    """cg_memory_stats: the peak covers what a growth needs (S_12 pancake with
    every layer kept holds all 12! packed states, 3.83 GB), and the bytes
    held go back down when the engine is closed."""
    import gc
    gc.collect()
    before = api.memory_stats(reset_peak=True)
    eng = api.Engine()
    r = eng.run(12, I.pancake(12), max_layers=512, keep_all_layers=True)
    assert sum(r.sizes) == 479001600
    during = api.memory_stats()
    assert during["peak_held_bytes"] >= before["held_bytes"] + 8 * 479001600
    assert during["held_bytes"] >= before["held_bytes"]
    eng.close()
    after = api.memory_stats()
    assert after["held_bytes"] <= before["held_bytes"] + (64 << 20)
    assert after["peak_held_bytes"] == during["peak_held_bytes"]
