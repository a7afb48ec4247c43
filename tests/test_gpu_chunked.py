"""Layers computed in key-range chunks (candidates larger than the memory
budget, forced small here through CG_CHUNK_CANDIDATES) against the oracle
and against the unchunked path. Tolerance: none (exact integers)."""

import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2509_19162_amd import _native as N  # noqa: E402
from paper_2509_19162_amd import api  # noqa: E402
from paper_2509_19162_amd import inputs as I  # noqa: E402


@pytest.fixture
def chunk_cap():
    old = os.environ.get("CG_CHUNK_CANDIDATES")

    def set_(v):
        if v is None:
            os.environ.pop("CG_CHUNK_CANDIDATES", None)
        else:
            os.environ["CG_CHUNK_CANDIDATES"] = str(v)

    yield set_
    set_(old)


@pytest.mark.parametrize("packed", [False, True])
@pytest.mark.parametrize("fam,n", [("pancake", 9), ("coxeter", 8), ("all_transpositions", 8), ("lrx", 10),
                                   ("star", 9)])
def test_chunked_growth_matches_oracle(fam, n, packed, chunk_cap, oracle_c):
    gens = I.family(fam, n)
    exp, rc, _ = oracle_c.growth(n, gens, max_layers=512)
    for cap in (20000, 300000):
        chunk_cap(cap)
        r = api.growth_ex(n, gens, max_layers=512, packed_sort=packed)
        assert r.status == rc == N.CG_OK
        assert r.sizes == exp


def test_chunked_layers_equal_unchunked_contents(chunk_cap):
    n, gens = 9, I.pancake(9)
    chunk_cap(None)
    ref = api.growth_ex(n, gens, max_layers=64, export_layers=362880)
    chunk_cap(7000)
    got = api.growth_ex(n, gens, max_layers=64, export_layers=362880)
    assert got.sizes == ref.sizes
    for a, b in zip(got.layers, ref.layers):
        assert np.array_equal(a, b)
    got_all = api.growth_ex(n, gens, max_layers=64, keep_all_layers=True, export_layers=362880)
    assert got_all.sizes == ref.sizes
    for a, b in zip(got_all.layers, ref.layers):
        assert np.array_equal(a, b)


def test_chunked_coset_start_and_stop_rules(chunk_cap, oracle_c):
    chunk_cap(5000)
    n = 12
    start = I.binary_central_state(n)
    gens = I.family("all_transpositions", n)
    r = api.growth_ex(n, gens, max_layers=64, start=start)
    exp, rc, _ = oracle_c.growth(n, gens, max_layers=64, start=start)
    assert r.sizes == exp and r.status == rc
    r = api.growth_ex(9, I.pancake(9), max_layers=512, max_frontier=5000)
    exp, rc, _ = oracle_c.growth(9, I.pancake(9), max_layers=512, max_frontier=5000)
    assert r.sizes == exp and r.status == rc == N.CG_TRUNCATED


def test_chunk_smaller_than_one_key_range_is_nomem(chunk_cap):
    chunk_cap(1)
    with pytest.raises(api.CGError) as e:
        api.growth_ex(7, I.pancake(7), max_layers=64)
    assert e.value.code == N.CG_E_NOMEM
