"""Batched growth (cg_growth_batch) against the oracle and against the same
jobs run alone. Tolerance: none (exact integers)."""

import json
import os

import pytest

pytestmark = pytest.mark.gpu

from golden_data import GOLDEN  # noqa: E402
from paper_2509_19162_amd import _native as N  # noqa: E402
from paper_2509_19162_amd import api  # noqa: E402
from paper_2509_19162_amd import inputs as I  # noqa: E402


def mixed_jobs(count, seed, n_lo=4, n_hi=9):
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


@pytest.mark.parametrize("seed", [1, 2])
def test_batch_matches_oracle(seed, oracle_c):
    jobs = mixed_jobs(96, seed)
    res = api.growth_batch(jobs, max_layers=512)
    for (n, gens), r in zip(jobs, res):
        exp, rc, _ = oracle_c.growth(n, gens, max_layers=512)
        assert r.status == rc == N.CG_OK
        assert r.sizes == exp
        assert r.states_expanded == sum(exp)


def test_batch_equals_alone_with_stop_rules(oracle_c):
    base = mixed_jobs(40, 3, 6, 9)
    jobs = []
    for i, (n, gens) in enumerate(base):
        mf = [None, 50, 1000][i % 3]
        ml = [None, 3, 9, None][i % 4]
        jobs.append((n, gens, mf, ml))
    res = api.growth_batch(jobs, max_layers=512)
    for (n, gens, mf, ml), r in zip(jobs, res):
        alone = api.growth_ex(n, gens, max_layers=ml or 512, max_frontier=mf)
        assert r.sizes == alone.sizes and r.status == alone.status
        exp, rc, _ = oracle_c.growth(n, gens, max_layers=ml or 512, max_frontier=mf or 0)
        assert r.sizes == exp and r.status == rc


def test_batch_degenerate_and_invalid_jobs():
    jobs = [(5, I.coxeter(5)), (4, [[0, 1, 2, 3]]), (3, [[0, 1, 1]]), (1, [[0]]), (6, I.lrx(6))]
    res = api.growth_batch(jobs)
    assert res[0].sizes == api.growth(5, I.coxeter(5))
    assert res[1].sizes == [1] and res[1].status == N.CG_OK
    assert res[2].status == N.CG_E_INVAL
    assert res[3].sizes == [1]
    assert res[4].sizes == api.growth(6, I.lrx(6))


def test_batch_of_one_large_job():
    res = api.growth_batch([(11, I.pancake(11))])
    assert res[0].sizes == api.growth(11, I.pancake(11))


def test_batch_small_groups_match(oracle_c):
    jobs = mixed_jobs(50, 5, 5, 8)
    res = api.growth_batch(jobs, max_active=7)
    for (n, gens), r in zip(jobs, res):
        assert r.sizes == oracle_c.growth(n, gens)[0]


def test_batch_workload_4096_matches_oracle():
    path = os.path.join(GOLDEN, "oracle_growth.json")
    if not os.path.exists(path):
        pytest.skip("oracle fixtures not generated")
    d = json.load(open(path))
    if "batch_4096" not in d:
        pytest.skip("batch fixture not generated")
    jobs = I.batch_jobs(4096)
    res = api.growth_batch(jobs, max_layers=512)
    exp = d["batch_4096"]["sizes"]
    bad = [i for i, r in enumerate(res) if r.sizes != exp[i]]
    assert not bad, bad[:10]


def test_batch_few_heavy_jobs_and_many_light(oracle_c):
    # heavy jobs (S_9 all transpositions) beside many light ones: the heavy
    # ones leave the one-workgroup engine; every result stays exact
    heavy = [(9, I.all_transpositions(9)), (9, I.pancake(9))]
    light = [(n, g) for n, g in [(6, I.coxeter(6)), (7, I.star(7)), (5, I.lrx(5))] * 5]
    jobs = heavy + light
    res = api.growth_batch(jobs, max_layers=512)
    for (n, gens), r in zip(jobs, res):
        assert r.sizes == oracle_c.growth(n, gens, max_layers=512)[0]


def test_batch_graph_replays_across_calls(oracle_c):
    """Repeated batches of one shape replay the small-job launch graph that
    the first one built, with the same results."""
    jobs = mixed_jobs(64, 7, 5, 9)
    first = api.growth_batch(jobs, max_layers=512)
    before = api.batch_info()
    again = [api.growth_batch(jobs, max_layers=512) for _ in range(3)]
    after = api.batch_info()
    assert after["calls"] == before["calls"] + 3
    assert after["graph_launches"] == before["graph_launches"] + 3
    assert after["graph_builds"] == before["graph_builds"]  # all three replayed
    for res in [first] + again:
        for (n, gens), r in zip(jobs, res):
            assert r.sizes == oracle_c.growth(n, gens, max_layers=512)[0]


def test_batch_autotuner_choices_are_kept_and_exact(oracle_c, tmp_path, monkeypatch):
    """The autotuner times engines, workgroup sizes, group sizes and the
    heavy-job split on the batch; its choices go to the tuning file and
    every result stays exact."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("CG_TUNE_CACHE", str(path))
    jobs = I.batch_jobs(4096)[:600]
    res = api.growth_batch(jobs, max_layers=512, tune=True)
    exp = _stored_batch()
    for i, r in enumerate(res):
        assert r.sizes == exp[i], i
    info = api.batch_info()
    assert info["tuned_classes"] >= 1 and info["heavy_split"] in (16.0, 64.0, 256.0)
    lines = path.read_text().split("\n")
    assert any(" class " in ln for ln in lines) and any(" heavy " in ln for ln in lines)
    res2 = api.growth_batch(jobs, max_layers=512, tune=True)  # the kept choices, no re-tuning
    assert [r.sizes for r in res2] == [r.sizes for r in res]


def _stored_batch():
    path = os.path.join(GOLDEN, "oracle_growth.json")
    if not os.path.exists(path):
        pytest.skip("oracle fixtures not generated")
    return json.load(open(path))["batch_4096"]["sizes"]


def test_release_frees_the_buffers_batches_keep(oracle_c):
    """cg_release_cached_memory also frees what batches keep between calls
    (the small-job runner's buffers and launch graph), so the device arena
    is freed (hipFree); the next batch builds its graph again and
    gives the same results."""
    import torch

    jobs = mixed_jobs(64, 7, 5, 10)
    api.growth_batch(jobs, max_layers=512)
    assert sum(api.growth(11, I.pancake(11))) == 39916800  # large buffers: the arena is reserved
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    api.release_cached_memory()
    free, total = torch.cuda.mem_get_info()
    assert free > total // 2, (free, total)
    before = api.batch_info()
    res = api.growth_batch(jobs, max_layers=512)
    assert api.batch_info()["graph_builds"] == before["graph_builds"] + 1
    for (n, gens), r in zip(jobs, res):
        assert r.sizes == oracle_c.growth(n, gens, max_layers=512)[0]
