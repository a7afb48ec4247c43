"""Directed generating sets (not closed under inverses) on the sort path:
every layer is taken against all visited states. Against the oracle (which
keeps its whole visited set) and the paper's directed diameters.
Tolerance: none (exact integers)."""

import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from golden_data import max_diameter_table  # noqa: E402
from paper_2509_19162_amd import _native as N  # noqa: E402
from paper_2509_19162_amd import api  # noqa: E402
from paper_2509_19162_amd import inputs as I  # noqa: E402


def random_directed(seed, n_lo, n_hi):
    r = I.rng_for(seed, seed=31)
    n = int(r.integers(n_lo, n_hi + 1))
    gens = [list(map(int, r.permutation(n))) for _ in range(int(r.integers(1, 4)))]
    return n, gens


@pytest.mark.parametrize("packed", [False, True])
@pytest.mark.parametrize("seed", range(8))
def test_directed_random_sets_match_oracle(seed, packed, oracle_c):
    n, gens = random_directed(seed, 3, 9)
    r = api.growth_ex(n, gens, max_layers=1024, allow_directed=True, packed_sort=packed)
    exp, rc, _ = oracle_c.growth(n, gens, max_layers=1024)
    assert r.status == rc and r.sizes == exp


@pytest.mark.parametrize("row", [r for r in max_diameter_table(directed=True) if r[0] <= 10],
                         ids=lambda r: f"n{r[0]}")
def test_directed_paper_diameters(row, oracle_c):
    n, diam, gens = row
    r = api.growth_ex(n, gens, max_layers=512, allow_directed=True)
    assert r.status == N.CG_OK
    assert len(r.sizes) - 1 == diam
    assert sum(r.sizes) == math.factorial(n)
    if n <= 9:
        assert r.sizes == oracle_c.growth(n, gens, max_layers=512)[0]


@pytest.mark.parametrize("n", range(5, 11))
def test_lx_diameter_formula(n):
    # LX (left shift and the swap of positions 0, 1): diameter (3n^2-8n+9)/4
    # for odd n and (3n^2-8n+12)/4 for even n (paper, LX case study)
    r = api.growth_ex(n, I.lx(n), max_layers=512, allow_directed=True)
    d = len(r.sizes) - 1
    assert d == ((3 * n * n - 8 * n + 9) // 4 if n % 2 else (3 * n * n - 8 * n + 12) // 4)
    assert sum(r.sizes) == math.factorial(n)
    assert r.sizes == api.growth_ex(n, I.lx(n), max_layers=512, allow_directed=True, bitmask=True).sizes


def test_directed_layer_contents_match_oracle(oracle_c):
    n, gens = 7, I.lx(7)
    r = api.growth_ex(n, gens, max_layers=512, allow_directed=True, keep_all_layers=True, export_layers=5040)
    sizes, rc, states = oracle_c.growth(n, gens, max_layers=512, with_states=True)
    assert r.sizes == sizes
    off = 0
    for layer, s in zip(r.layers, sizes):
        exp = states[off: off + s]
        off += s
        key = lambda a: sorted(map(tuple, np.asarray(a).tolist()))
        assert key(layer) == key(exp)


def test_directed_chunked_and_coset_start(oracle_c):
    old = os.environ.get("CG_CHUNK_CANDIDATES")
    os.environ["CG_CHUNK_CANDIDATES"] = "3000"
    try:
        n, gens = random_directed(101, 8, 9)
        r = api.growth_ex(n, gens, max_layers=1024, allow_directed=True)
        assert r.sizes == oracle_c.growth(n, gens, max_layers=1024)[0]
    finally:
        if old is None:
            os.environ.pop("CG_CHUNK_CANDIDATES", None)
        else:
            os.environ["CG_CHUNK_CANDIDATES"] = old
    n = 12
    start = I.binary_central_state(n)
    r = api.growth_ex(n, I.lx(n), max_layers=512, start=start, allow_directed=True)
    exp, rc, _ = oracle_c.growth(n, I.lx(n), max_layers=512, start=start)
    assert r.sizes == exp and r.status == rc


def test_directed_stop_rules(oracle_c):
    gens = I.lx(9)
    r = api.growth_ex(9, gens, max_layers=10, allow_directed=True)
    exp, rc, _ = oracle_c.growth(9, gens, max_layers=10)
    assert r.sizes == exp and r.status == rc == N.CG_TRUNCATED
    r = api.growth_ex(9, gens, max_layers=512, max_frontier=2000, allow_directed=True)
    exp, rc, _ = oracle_c.growth(9, gens, max_layers=512, max_frontier=2000)
    assert r.sizes == exp and r.status == rc
