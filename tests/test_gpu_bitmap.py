"""Rank-space bitmap engines against the oracle: the bitmask engine (one job
over the device, CG_BITMASK) and the small-job engine (one workgroup per
job inside cg_growth_batch). Tolerance: none (exact integers)."""

import json
import math
import os

import pytest

pytestmark = pytest.mark.gpu

from golden_data import GOLDEN, max_diameter_table  # noqa: E402
from paper_2509_19162_amd import _native as N  # noqa: E402
from paper_2509_19162_amd import api  # noqa: E402
from paper_2509_19162_amd import inputs as I  # noqa: E402

FAMILIES = ["coxeter", "pancake", "lrx", "star", "all_transpositions", "reversals"]


def mahonian(n):
    poly = [1]
    for i in range(1, n + 1):
        nxt = [0] * (len(poly) + i - 1)
        for a, c in enumerate(poly):
            for b in range(i):
                nxt[a + b] += c
        poly = nxt
    return poly


def stirling_first(n):
    # c(n, k) by the recurrence c(n+1, k) = n c(n, k) + c(n, k-1)
    row = [1]
    for m in range(n):
        new = [0] * (len(row) + 1)
        for k, c in enumerate(row):
            new[k] += m * c
            new[k + 1] += c
        row = new
    return [row[n - m] for m in range(n)]


@pytest.mark.parametrize("fam", FAMILIES)
@pytest.mark.parametrize("n", [3, 5, 7, 9])
def test_bitmask_families_match_oracle(fam, n, oracle_c):
    gens = I.family(fam, n)
    r = api.growth_ex(n, gens, max_layers=512, bitmask=True)
    exp, rc, _ = oracle_c.growth(n, gens, max_layers=512)
    assert r.status == rc == N.CG_OK
    assert r.sizes == exp
    assert r.states_expanded == sum(exp)


@pytest.mark.parametrize("n", [10, 11, 12])
def test_bitmask_closed_forms(n):
    assert api.growth_ex(n, I.coxeter(n), max_layers=512, bitmask=True).sizes == mahonian(n)
    if n <= 11:
        assert api.growth_ex(n, I.all_transpositions(n), max_layers=64, bitmask=True).sizes == stirling_first(n)


def test_bitmask_pancake12_matches_stored_oracle():
    path = os.path.join(GOLDEN, "oracle_growth.json")
    if not os.path.exists(path):
        pytest.skip("oracle fixtures not generated")
    exp = json.load(open(path))["pancake_12"]["sizes"]
    a = api.growth_ex(12, I.pancake(12), max_layers=64, bitmask=True)
    assert a.sizes == exp and a.status == N.CG_OK


def test_bitmask_n13_coxeter_prefix():
    # 64-bit ranks (13! > 2^32); the first 30 layers of the Mahonian numbers
    r = api.growth_ex(13, I.coxeter(13), max_layers=30, bitmask=True)
    assert r.status == N.CG_TRUNCATED
    assert r.sizes == mahonian(13)[:30]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bitmask_random_sets_and_starts(seed, oracle_c):
    r0 = I.rng_for(seed, seed=77)
    n = int(r0.integers(5, 10))
    gens = I.random_perms_with_inverses(n, int(r0.integers(1, 4)), r0)
    start = [int(x) for x in r0.permutation(n)]
    r = api.growth_ex(n, gens, max_layers=512, start=start, bitmask=True)
    exp, rc, _ = oracle_c.growth(n, gens, max_layers=512, start=start)
    assert r.sizes == exp and r.status == rc


@pytest.mark.parametrize("row", [r for r in max_diameter_table(directed=True) if r[0] <= 13],
                         ids=lambda r: f"n{r[0]}")
def test_bitmask_directed_paper_diameters(row, oracle_c):
    n, diam, gens = row
    r = api.growth_ex(n, gens, max_layers=512, allow_directed=True, bitmask=True)
    assert r.status == N.CG_OK
    assert len(r.sizes) - 1 == diam
    assert sum(r.sizes) == math.factorial(n)
    if n <= 9:
        assert r.sizes == oracle_c.growth(n, gens, max_layers=512)[0]


def test_bitmask_stop_rules(oracle_c):
    gens = I.pancake(9)
    r = api.growth_ex(9, gens, max_layers=4, bitmask=True)
    assert r.status == N.CG_TRUNCATED and r.sizes == oracle_c.growth(9, gens, max_layers=4)[0]
    r = api.growth_ex(9, gens, max_layers=512, max_frontier=1000, bitmask=True)
    exp, rc, _ = oracle_c.growth(9, gens, max_layers=512, max_frontier=1000)
    assert r.status == rc == N.CG_TRUNCATED and r.sizes == exp


def test_bitmask_rejects_what_it_cannot_do():
    with pytest.raises(api.CGError):
        api.growth_ex(15, I.coxeter(15), max_layers=4, bitmask=True)
    with pytest.raises(api.CGError):
        api.growth_ex(8, I.coxeter(8), bitmask=True, export_layers=100)
    with pytest.raises(api.CGError):  # repeated entries: not a permutation start
        api.growth_ex(6, I.coxeter(6), start=[0, 0, 0, 1, 1, 1], bitmask=True)


def test_bitmask_single_state_and_trivial():
    assert api.growth_ex(1, [[0]], bitmask=True).sizes == [1]
    assert api.growth_ex(2, [[1, 0]], bitmask=True).sizes == [1, 1]


# ---- small-job engine (inside cg_growth_batch) --------------------------------


def mixed_small_jobs(count, seed, n_lo, n_hi):
    jobs = []
    for j in range(count):
        r = I.rng_for(j, seed=seed)
        n = int(r.integers(n_lo, n_hi + 1))
        kind = int(r.integers(0, 3))
        if kind == 0:
            gens = I.random_perms_with_inverses(n, int(r.integers(1, 4)), r)
        elif kind == 1:
            gens = I.random_involutions(n, int(r.integers(2, 4)), r)
        else:
            gens = I.family(["coxeter", "pancake", "lrx", "star"][j % 4], n)
        jobs.append((n, gens))
    return jobs


@pytest.fixture
def wg_max_n():
    old = os.environ.get("CG_WG_MAX_N")

    def set_(v):
        os.environ["CG_WG_MAX_N"] = str(v)

    yield set_
    if old is None:
        os.environ.pop("CG_WG_MAX_N", None)
    else:
        os.environ["CG_WG_MAX_N"] = old


@pytest.mark.parametrize("limit", [0, 8, 10])
def test_small_job_engine_matches_oracle(limit, wg_max_n, oracle_c):
    wg_max_n(limit)
    jobs = mixed_small_jobs(160, 11, 3, 10)
    res = api.growth_batch(jobs, max_layers=512)
    for (n, gens), r in zip(jobs, res):
        exp, rc, _ = oracle_c.growth(n, gens, max_layers=512)
        assert r.status == rc == N.CG_OK, (n, gens)
        assert r.sizes == exp, (n, gens)
        # a set of identities expands nothing
        trivial = all(list(g) == list(range(n)) for g in gens)
        assert r.states_expanded == (0 if trivial else sum(exp))


def test_small_job_engine_stop_rules(wg_max_n, oracle_c):
    wg_max_n(10)
    base = mixed_small_jobs(60, 12, 5, 10)
    jobs = []
    for i, (n, gens) in enumerate(base):
        mf = [None, 50, 1000][i % 3]
        ml = [None, 3, 9, None][i % 4]
        jobs.append((n, gens, mf, ml))
    res = api.growth_batch(jobs, max_layers=512)
    for (n, gens, mf, ml), r in zip(jobs, res):
        exp, rc, _ = oracle_c.growth(n, gens, max_layers=ml or 512, max_frontier=mf or 0)
        assert r.sizes == exp and r.status == rc


def test_small_job_engine_directed_sets(wg_max_n, oracle_c):
    wg_max_n(10)
    jobs = []
    for j in range(40):
        r = I.rng_for(j, seed=13)
        n = int(r.integers(3, 10))
        gens = [list(map(int, r.permutation(n))) for _ in range(int(r.integers(1, 3)))]
        jobs.append((n, gens))
    jobs += [(n, g) for n, _, g in max_diameter_table(directed=True) if n <= 9]
    res = api.growth_batch(jobs, max_layers=512, allow_directed=True)
    for (n, gens), r in zip(jobs, res):
        exp, rc, _ = oracle_c.growth(n, gens, max_layers=512)
        assert r.status == rc and r.sizes == exp, (n, gens)


def test_small_job_engine_repeat_and_tuned(wg_max_n, oracle_c):
    # the same batch twice (graph replay) and with the autotuner
    wg_max_n(9)
    jobs = mixed_small_jobs(300, 14, 6, 9)
    exp = [oracle_c.growth(n, g, max_layers=512)[0] for n, g in jobs]
    for tune in (False, False, True):
        res = api.growth_batch(jobs, max_layers=512, tune=tune)
        assert [r.sizes for r in res] == exp


def test_small_job_flag_on_engine_replays_graph(oracle_c):
    eng = api.Engine()
    for n, fam in [(8, "coxeter"), (8, "coxeter"), (9, "pancake"), (7, "lrx"), (8, "coxeter")]:
        gens = I.family(fam, n)
        r = eng.run(n, gens, max_layers=512, small_job=True)
        exp, rc, _ = oracle_c.growth(n, gens, max_layers=512)
        assert r.status == rc and r.sizes == exp
    r = eng.run(8, I.coxeter(8), max_layers=5, small_job=True)
    assert r.status == N.CG_TRUNCATED and r.sizes == oracle_c.growth(8, I.coxeter(8), max_layers=5)[0]
    with pytest.raises(api.CGError):
        eng.run(11, I.coxeter(11), small_job=True)
    eng.close()


def test_bitmask_full_s14_coxeter_is_mahonian():
    # the whole of S_14 (8.7e10 states, 92 layers) on one device: about 30 s
    r = api.growth_ex(14, I.coxeter(14), max_layers=128, bitmask=True)
    assert r.status == N.CG_OK
    assert r.sizes == mahonian(14)
