"""Binary states: Schreier coset graphs of a 0/1 start vector with one bit
per entry (CG_BINARY_STATE; implied for n > 16, up to 64), against the
oracle (Python set BFS over tuples), the 4-bit path, closed forms and
conjugation invariance. Tolerance: none (exact integers)."""

import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from golden_data import binary_coset_growth  # noqa: E402
from oracle import bfs_set  # noqa: E402
from paper_2509_19162_amd import _native as N  # noqa: E402
from paper_2509_19162_amd import api  # noqa: E402
from paper_2509_19162_amd import inputs as I  # noqa: E402


def random_binary_start(n, rng):
    z = int(rng.integers(1, n))
    v = np.array([0] * z + [1] * (n - z), dtype=np.uint8)
    rng.shuffle(v)
    return [int(x) for x in v]


@pytest.mark.parametrize("n", [5, 8, 11, 16])
@pytest.mark.parametrize("fam", ["reversals", "transposons", "coxeter", "lrx", "star"])
def test_binary_equals_4bit_path(n, fam):
    """n <= 16: the same growth and layer contents with one bit per entry as
    with four."""
    gens = I.family(fam, n)
    for start in (I.binary_central_state(n), random_binary_start(n, np.random.default_rng([n, 3]))):
        a = api.growth_ex(n, gens, start=start, max_layers=512, export_layers=1 << 16)
        b = api.growth_ex(n, gens, start=start, max_layers=512, export_layers=1 << 16, binary_state=True)
        assert a.sizes == b.sizes and a.status == b.status
        for la, lb in zip(a.layers, b.layers):
            assert np.array_equal(la, lb)


@pytest.mark.parametrize("n,fam", [(17, "coxeter"), (17, "reversals"), (18, "star"), (18, "lrx"),
                                   (20, "lrx"), (20, "coxeter")])
def test_binary_matches_oracle(n, fam):
    gens = I.family(fam, n)
    start = I.binary_central_state(n)
    r = api.growth_ex(n, gens, start=start, max_layers=512)
    assert r.sizes == bfs_set.growth(n, gens, start=start)
    assert r.status == N.CG_OK
    assert sum(r.sizes) == math.comb(n, n // 2)


@pytest.mark.parametrize("n", [17, 19])
def test_binary_random_sets_and_starts_match_oracle(n):
    rng = np.random.default_rng([I.SEED, n])
    for _ in range(3):
        gens = I.random_perms_with_inverses(n, int(rng.integers(1, 4)), rng)
        start = random_binary_start(n, rng)
        r = api.growth_ex(n, gens, start=start, max_layers=512)
        assert r.sizes == bfs_set.growth(n, gens, start=start)


@pytest.mark.parametrize("n", [17, 21, 24, 27, 28])
def test_reversal_cosets_closed_form(n):
    """Reversals on the central binary state: C(m,k)^2 (n = 2m) or
    C(m,k) C(m+1,k) (n = 2m+1), the closed form of the paper's section on
    binary cosets, checked by the oracle for n <= 16 elsewhere."""
    r = api.growth_ex(n, I.reversals(n), start=I.binary_central_state(n), max_layers=64)
    assert r.sizes == binary_coset_growth(n)


@pytest.mark.parametrize("n", [17, 20, 22])
def test_transposon_cosets_closed_form(n):
    r = api.growth_ex(n, I.transposons(n), start=I.binary_central_state(n), max_layers=64)
    assert r.sizes == binary_coset_growth(n)


@pytest.mark.parametrize("n,fam", [(40, "lrx"), (40, "coxeter"), (64, "lrx"), (64, "star"), (33, "reversals")])
def test_binary_large_n_truncated_matches_oracle(n, fam):
    """n up to 64: the first layers (stopped at the first one above 3000
    states) equal the oracle's, state by state."""
    gens = I.family(fam, n)
    start = random_binary_start(n, np.random.default_rng([n, 11]))
    r = api.growth_ex(n, gens, start=start, max_layers=512, max_frontier=3000, export_layers=1 << 16)
    layers, complete = bfs_set.bfs_layers(n, gens, max_frontier=3000, start=start)
    assert r.sizes == [len(x) for x in layers]
    assert r.status == (N.CG_OK if complete else N.CG_TRUNCATED)
    for got, exp in zip(r.layers, layers):
        assert np.array_equal(got, np.array(sorted(exp), dtype=np.uint8).reshape(-1, n))


def test_binary_full_growth_n32_conjugation_invariant():
    """n = 32, LRX from the central state: every state of the orbit
    (C(32,16)) is reached, and conjugating the generators by a random h
    while starting from s.h gives the same growth (t -> t.h maps one BFS
    onto the other)."""
    n = 32
    s = I.binary_central_state(n)
    gens = I.lrx(n)
    a = api.growth_ex(n, gens, start=s, max_layers=2048)
    assert a.status == N.CG_OK and sum(a.sizes) == math.comb(32, 16)
    h = [int(x) for x in np.random.default_rng(32).permutation(n)]
    hinv = [0] * n
    for i, v in enumerate(h):
        hinv[v] = i
    # psi(t) = t.h maps t.g to psi(t).g' with g'[i] = hinv[g[h[i]]] (gather
    # action t.g[i] = t[g[i]]): the BFS from s.h under the g' is the image
    # of the BFS from s under the g
    conj = [[hinv[g[h[i]]] for i in range(n)] for g in gens]
    sh = [s[h[i]] for i in range(n)]
    b = api.growth_ex(n, conj, start=sh, max_layers=2048)
    assert b.sizes == a.sizes


def test_binary_directed_stop_rules_and_keep_all():
    n = 18
    s = I.binary_central_state(n)
    lx = I.lx(n)
    r = api.growth_ex(n, lx, start=s, max_layers=512, allow_directed=True)
    assert r.sizes == bfs_set.growth(n, lx, start=s)
    for kw in ({"max_layers": 5}, {"max_frontier": 500}):
        r = api.growth_ex(n, I.coxeter(n), start=s, **kw)
        exp = bfs_set.growth(n, I.coxeter(n), start=s, **kw)
        assert r.sizes == exp and r.status == N.CG_TRUNCATED
    k = api.growth_ex(n, I.coxeter(n), start=s, max_layers=512, keep_all_layers=True)
    assert k.sizes == bfs_set.growth(n, I.coxeter(n), start=s)


def test_batches_and_queue_refuse_binary_states():
    n = 20
    s = I.binary_central_state(n)
    # a batch job carries no start vector: n > 16 cannot be a binary state
    res = api.growth_batch([(n, I.lrx(n)), (6, I.coxeter(6))], max_layers=64)
    assert res[0].status == N.CG_E_INVAL and res[1].sizes == api.growth(6, I.coxeter(6))
    with api.GrowthQueue() as q:
        with pytest.raises(api.CGError) as e:
            q.submit(n, I.lrx(n), start=s)
        assert e.value.code == N.CG_E_UNSUPPORTED


def test_binary_chunked_layers(monkeypatch):
    """Key-range chunks of binary candidates (forced small) give the same
    layers: reversal cosets against the closed form, LRX against the
    oracle."""
    n = 24
    monkeypatch.setenv("CG_CHUNK_CANDIDATES", "50000000")
    r = api.growth_ex(n, I.reversals(n), start=I.binary_central_state(n), max_layers=64)
    assert r.sizes == binary_coset_growth(n)
    monkeypatch.setenv("CG_CHUNK_CANDIDATES", "5000")
    s = I.binary_central_state(20)
    r = api.growth_ex(20, I.lrx(20), start=s, max_layers=4096, export_layers=200_000)
    layers, _ = bfs_set.bfs_layers(20, I.lrx(20), start=s)
    assert r.sizes == [len(x) for x in layers]
    for got, exp in zip(r.layers, layers):
        assert np.array_equal(got, np.array(sorted(exp), dtype=np.uint8).reshape(-1, 20))


def test_reversal_cosets_n30_chunked_by_memory():
    """n = 30: 435 reversals on the central state; the largest layer's
    1.8e10 candidates do not fit at once and run in key-range chunks."""
    n = 30
    r = api.growth_ex(n, I.reversals(n), start=I.binary_central_state(n), max_layers=64)
    assert r.sizes == binary_coset_growth(n)
