"""cg_growth_batch_noalloc (the small-job engine on the library's static
device array) against cg_growth_batch on the same jobs: two calls in a row,
the second smaller, each result equal bit for bit. Tolerance: none."""

import json
import os

import pytest

pytestmark = pytest.mark.gpu

from golden_data import GOLDEN  # noqa: E402
from paper_2509_19162_amd import _native as N  # noqa: E402
from paper_2509_19162_amd import api  # noqa: E402
from paper_2509_19162_amd import inputs as I  # noqa: E402


def _mixed(count, seed, n_lo, n_hi):
    jobs = []
    for j in range(count):
        r = I.rng_for(j, seed=seed)
        n = int(r.integers(n_lo, n_hi + 1))
        kind = j % 4
        if kind == 0:
            gens = I.random_perms_with_inverses(n, int(r.integers(1, 4)), r)
        elif kind == 1:
            gens = I.random_involutions(n, int(r.integers(2, 4)), r)
        elif kind == 2:
            gens = I.family(["coxeter", "pancake", "lrx", "star"][(j // 4) % 4], n)
        else:
            gens = I.lx(n)  # not closed under inverses
        jobs.append((n, gens, None, [None, 4, None][j % 3]))
    return jobs


def _same(a, b):
    assert len(a) == len(b)
    for i, (x, y) in enumerate(zip(a, b)):
        assert (x.status, x.sizes, x.states_expanded, x.candidates) == (
            y.status, y.sizes, y.states_expanded, y.candidates), i


def test_noalloc_matches_batch_twice_second_smaller(oracle_c):
    print("noalloc call 1: 4096 jobs of S_7..S_10 (max_layers 512)", flush=True)
    jobs = I.batch_jobs(4096)
    got = api.growth_batch_noalloc(jobs, max_layers=512)
    ref = api.growth_batch(jobs, max_layers=512)
    _same(got, ref)
    path = os.path.join(GOLDEN, "oracle_growth.json")
    if os.path.exists(path):
        d = json.load(open(path))
        if "batch_4096" in d:
            exp = d["batch_4096"]["sizes"]
            assert [r.sizes for r in got] == exp
    print("noalloc call 2: 300 mixed jobs of S_4..S_9, directed ones included", flush=True)
    jobs = _mixed(300, 11, 4, 9)
    got = api.growth_batch_noalloc(jobs, allow_directed=True)
    ref = api.growth_batch(jobs, allow_directed=True)
    _same(got, ref)
    for (n, gens, mf, ml), r in zip(jobs, got):
        exp, rc, _ = oracle_c.growth(n, gens, max_layers=ml or 256)
        assert r.sizes == exp and r.status == rc
    print("noalloc call 3: 40 jobs of S_3..S_8 (no device slots)", flush=True)
    jobs = _mixed(40, 12, 3, 8)
    got = api.growth_batch_noalloc(jobs, allow_directed=True)
    ref = api.growth_batch(jobs, allow_directed=True)
    _same(got, ref)


def test_noalloc_bad_rows_fail_their_own_job():
    res = api.growth_batch_noalloc([(4, I.coxeter(4)), (3, [[0, 1, 1]]), (1, [[0]]), (10, I.star(10))])
    assert res[0].sizes == [1, 3, 5, 6, 5, 3, 1]
    assert res[1].status == N.CG_E_INVAL
    assert res[2].sizes == [1] and res[2].status == N.CG_OK
    assert res[3].sizes == api.growth(10, I.star(10))
