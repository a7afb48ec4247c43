"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value comes
from a closed form, a value printed in the paper (``tests/golden``), or an
invariant of Cayley graphs.
"""

import math

import pytest

from golden_data import (
    binary_coset_growth,
    lx_diameter,
    mahonian,
    max_diameter_table,
    reversal_sphere2,
    transposition_growth,
)
from oracle import bfs_set
from paper_2509_19162_amd import inputs as I


def both(n, gens, oracle_c, **kw):
    """Growth from the Python oracle (small n) and the C oracle; they must agree."""
    sizes_c, rc, _ = oracle_c.growth(n, gens, **kw)
    if math.factorial(n) <= 40320:
        kw2 = {}
        if "start" in kw:
            kw2["start"] = kw["start"]
        assert bfs_set.growth(n, gens, **kw2) == sizes_c
    return sizes_c, rc


@pytest.mark.parametrize("n", range(2, 10))
def test_coxeter_is_mahonian(n, oracle_c):
    sizes, rc = both(n, I.coxeter(n), oracle_c)
    assert rc == 0
    assert sizes == mahonian(n)
    assert len(sizes) - 1 == n * (n - 1) // 2
    assert sizes[-1] == 1
    assert sizes == sizes[::-1]


@pytest.mark.parametrize("n", range(2, 10))
def test_all_transpositions_is_stirling(n, oracle_c):
    sizes, rc = both(n, I.all_transpositions(n), oracle_c)
    assert rc == 0
    assert sizes == transposition_growth(n)
    assert sizes[-1] == math.factorial(n - 1)


@pytest.mark.parametrize("n", range(2, 10))
def test_star_diameter(n, oracle_c):
    sizes, _ = both(n, I.star(n), oracle_c)
    assert len(sizes) - 1 == (3 * (n - 1)) // 2
    assert sum(sizes) == math.factorial(n)


@pytest.mark.parametrize("n", range(3, 10))
def test_cyclic_coxeter_diameter(n, oracle_c):
    sizes, _ = both(n, I.cyclic_coxeter(n), oracle_c)
    assert len(sizes) - 1 == (n * n) // 4
    assert sum(sizes) == math.factorial(n)


@pytest.mark.parametrize("n", range(4, 11))
def test_lrx_diameter(n, oracle_c):
    # conjectured n(n-1)/2; n = 3 is degenerate (diameter 2) and not covered
    sizes, _ = both(n, I.lrx(n), oracle_c)
    assert len(sizes) - 1 == n * (n - 1) // 2
    assert sum(sizes) == math.factorial(n)


@pytest.mark.parametrize("n", range(5, 11))
def test_lx_directed_diameter(n, oracle_c):
    # conjectured quasi-polynomial; it holds from n = 5 (n = 3, 4 are below its range)
    sizes, _ = both(n, I.lx(n), oracle_c)
    assert len(sizes) - 1 == lx_diameter(n)
    assert sum(sizes) == math.factorial(n)


@pytest.mark.parametrize("n", range(3, 10))
def test_reversal_spheres(n, oracle_c):
    sizes, _ = both(n, I.reversals(n), oracle_c)
    assert sizes[1] == math.comb(n, 2)
    assert sizes[2] == reversal_sphere2(n)
    assert len(sizes) - 1 == n - 1
    assert sizes[-1] == 2
    assert sum(sizes) == math.factorial(n)


@pytest.mark.parametrize("n", range(3, 10))
def test_transposon_diameter(n, oracle_c):
    sizes, _ = both(n, I.transposons(n), oracle_c)
    assert len(sizes) - 1 == (n + 2) // 2  # ceil((n+1)/2)
    assert sum(sizes) == math.factorial(n)


@pytest.mark.parametrize("n", range(3, 9))
def test_three_cycles_alternating(n, oracle_c):
    sizes, _ = both(n, I.three_cycles(n), oracle_c)
    assert sum(sizes) == math.factorial(n) // 2
    assert len(sizes) - 1 == n // 2


@pytest.mark.parametrize("row", max_diameter_table(directed=False), ids=lambda r: f"n{r[0]}")
def test_paper_max_diameter_undirected(row, oracle_c):
    n, diam, gens = row
    if n > 10:
        pytest.skip("S_11 and larger are pinned on the GPU path only (oracle RAM/time)")
    sizes, rc = both(n, gens, oracle_c)
    assert rc == 0
    assert len(sizes) - 1 == diam
    assert sum(sizes) == math.factorial(n)


@pytest.mark.parametrize("row", max_diameter_table(directed=True), ids=lambda r: f"n{r[0]}")
def test_paper_max_diameter_directed(row, oracle_c):
    n, diam, gens = row
    if n > 10:
        pytest.skip("S_11 and larger are out of the oracle's budget in the CPU suite")
    sizes, rc = both(n, gens, oracle_c)
    assert rc == 0
    assert len(sizes) - 1 == diam
    assert sum(sizes) == math.factorial(n)


@pytest.mark.parametrize("fam", ["reversals", "transposons"])
@pytest.mark.parametrize("n", range(2, 13))
def test_binary_coset_growth(fam, n, oracle_c):
    start = I.binary_central_state(n)
    sizes, rc = both(n, I.family(fam, n), oracle_c, start=start)
    assert rc == 0
    assert sizes == binary_coset_growth(n)
    assert len(sizes) - 1 == n // 2
    assert sum(sizes) == math.comb(n, n // 2)


def test_first_layer_counts_distinct_generators(oracle_c):
    gens = I.coxeter(6) + I.coxeter(6)[:2] + [list(range(6))]
    sizes, _ = both(6, gens, oracle_c)
    assert sizes[1] == 5


def test_stop_rules(oracle_c):
    # max_layers records exactly that many layers and reports truncation
    sizes, rc, _ = oracle_c.growth(8, I.coxeter(8), max_layers=5)
    assert sizes == mahonian(8)[:5] and rc == 1
    # max_frontier: the first layer larger than the limit is recorded, then stop
    sizes, rc, _ = oracle_c.growth(8, I.coxeter(8), max_frontier=100)
    m = mahonian(8)
    first_big = next(i for i, v in enumerate(m) if v > 100)
    assert sizes == m[: first_big + 1] and rc == 1
    assert bfs_set.growth(8, I.coxeter(8), max_frontier=100) == sizes
    assert bfs_set.growth(8, I.coxeter(8), max_layers=5) == m[:5]
    # n = 1: one state, complete
    assert oracle_c.growth(1, [[0]])[:2] == ([1], 0)
