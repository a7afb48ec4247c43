"""Pins of the oracle against computations that share none of its logic.

* word enumeration: the ball of radius m is the set of products of all words
  of length <= m, so gamma(m) = |W_<=m| - |W_<=m-1| (definition of the word
  metric; no frontier, no visited set);
* scipy's graph shortest paths on the explicitly built Cayley graph (a
  library routine on the adjacency the paper describes: an edge joins v and
  v.g);
* invariants of Cayley graphs: growth does not depend on the start vertex,
  conjugating all generators gives an isomorphic graph, S and S^-1 give the
  same growth.

A last group plants plausible mistakes in copies of the BFS and checks that
the pins reject every one of them.
"""

import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

from golden_data import mahonian, transposition_growth
from oracle import bfs_set
from paper_2509_19162_amd import inputs as I


def word_ball_growth(n, gens, max_len):
    """gamma(m) from the sets of products of all words of length <= m."""
    e = tuple(range(n))
    ball = {e}
    out = [1]
    for m in range(1, max_len + 1):
        words = set()
        for w in itertools.product(range(len(gens)), repeat=m):
            s = e
            for gi in w:
                s = tuple(s[gens[gi][i]] for i in range(n))
            words.add(s)
        new_ball = ball | words
        if len(new_ball) == len(ball):
            break
        out.append(len(new_ball) - len(ball))
        ball = new_ball
    return out


def scipy_growth(n, gens, start=None, directed=False):
    """Growth by scipy shortest paths on the explicit Cayley graph of S_n."""
    perms = list(itertools.permutations(range(n)))
    index = {p: i for i, p in enumerate(perms)}
    rows, cols = [], []
    for p in perms:
        for g in gens:
            q = tuple(p[g[i]] for i in range(n))
            rows.append(index[p])
            cols.append(index[q])
    N = len(perms)
    A = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(N, N))
    src = index[tuple(range(n)) if start is None else tuple(start)]
    d = shortest_path(A, directed=directed, unweighted=True, indices=src)
    d = d[np.isfinite(d)].astype(int)
    return list(np.bincount(d))


def random_gens(n, m, seed):
    rng = np.random.default_rng(seed)
    perms = [list(map(int, rng.permutation(n))) for _ in range(m)]
    return perms + [I.inverse(p) for p in perms]


@pytest.mark.parametrize(
    "n,gens,max_len",
    [
        (3, I.coxeter(3), 4),
        (4, I.coxeter(4), 7),
        (4, I.lrx(4), 7),
        (4, I.pancake(4), 5),
        (4, I.star(4), 5),
        (5, I.pancake(5), 6),
        (4, random_gens(4, 2, 1), 7),
        (5, random_gens(5, 1, 2), 9),
    ],
)
def test_oracle_matches_word_enumeration(n, gens, max_len, oracle_c):
    expected = word_ball_growth(n, gens, max_len)
    got = bfs_set.growth(n, gens)
    assert got[: len(expected)] == expected
    if len(expected) <= max_len:  # enumeration reached the whole group
        assert got == expected
    assert oracle_c.growth(n, gens)[0] == got


FAMS = ["coxeter", "cyclic_coxeter", "all_transpositions", "star", "pancake", "lrx",
        "reversals", "transposons", "three_cycles"]


@pytest.mark.parametrize("fam", FAMS)
@pytest.mark.parametrize("n", [5, 6, 7])
def test_oracle_matches_scipy_graph_bfs(fam, n, oracle_c):
    gens = I.family(fam, n)
    expected = scipy_growth(n, gens)
    assert bfs_set.growth(n, gens) == expected
    assert oracle_c.growth(n, gens)[0] == expected


@pytest.mark.parametrize("seed", range(6))
def test_oracle_matches_scipy_random_sets(seed, oracle_c):
    n = 5 + seed % 3
    gens = random_gens(n, 1 + seed % 3, seed)
    expected = scipy_growth(n, gens)
    assert bfs_set.growth(n, gens) == expected
    assert oracle_c.growth(n, gens)[0] == expected


@pytest.mark.parametrize("n", [5, 6])
def test_oracle_directed_matches_scipy(n, oracle_c):
    gens = I.lx(n)
    expected = scipy_growth(n, gens, directed=True)
    assert bfs_set.growth(n, gens) == expected
    assert oracle_c.growth(n, gens)[0] == expected


@pytest.mark.parametrize("seed", range(4))
def test_oracle_layer_contents_agree(seed, oracle_c):
    n = 6 + seed % 3
    gens = random_gens(n, 2, 100 + seed)
    layers, complete = bfs_set.bfs_layers(n, gens)
    sizes, rc, states = oracle_c.growth(n, gens, with_states=True)
    assert complete and rc == 0
    assert sizes == [len(x) for x in layers]
    off = 0
    for layer, sz in zip(layers, sizes):
        got = {tuple(int(v) for v in r) for r in states[off:off + sz]}
        assert got == set(layer)
        off += sz


@pytest.mark.parametrize("seed", range(5))
def test_start_vertex_conjugation_and_inverse_invariance(seed, oracle_c):
    rng = np.random.default_rng(500 + seed)
    n = 6 + seed % 3
    gens = random_gens(n, 2, 700 + seed)
    base = oracle_c.growth(n, gens)[0]
    start = [int(x) for x in rng.permutation(n)]
    assert oracle_c.growth(n, gens, start=start)[0] == base
    h = [int(x) for x in rng.permutation(n)]
    hinv = I.inverse(h)
    conj = [I.compose(I.compose(hinv, g), h) for g in gens]
    assert oracle_c.growth(n, conj)[0] == base
    inv = [I.inverse(g) for g in gens]
    assert oracle_c.growth(n, inv)[0] == base
    shuffled = [gens[i] for i in rng.permutation(len(gens))] + gens[:1]
    assert oracle_c.growth(n, shuffled)[0] == base


# --- planted mistakes: each must be caught by a pin ---------------------------

def _bfs_variant(n, gens, mistake):
    e = tuple(range(n))
    visited = {e}
    layers = [[e]]
    while len(layers) < 200:  # a wrong window can cycle on directed sets
        nxt = []
        seen_here = set()
        cur_set = set(layers[-1])
        prev = set(layers[-2]) if len(layers) > 1 else set()
        for s in layers[-1]:
            for g in gens:
                if mistake == "scatter_wrong_index":
                    t = tuple(s[g[g[i]]] for i in range(n))
                else:
                    t = tuple(s[g[i]] for i in range(n))
                if mistake == "no_dedup_within_layer":
                    if t not in visited:
                        nxt.append(t)
                    continue
                if mistake == "only_previous_layer":
                    if t in prev or t in cur_set or t in seen_here:
                        continue
                    seen_here.add(t)
                    nxt.append(t)
                    continue
                if t not in visited:
                    visited.add(t)
                    nxt.append(t)
        if mistake == "no_dedup_within_layer":
            visited.update(nxt)
        if not nxt:
            break
        layers.append(nxt)
    sizes = [len(x) for x in layers]
    if mistake == "drop_layer_zero":
        sizes = sizes[1:]
    return sizes


@pytest.mark.parametrize(
    "mistake", ["scatter_wrong_index", "no_dedup_within_layer", "drop_layer_zero"]
)
def test_pins_reject_planted_mistakes(mistake):
    n = 6
    caught = (
        _bfs_variant(n, I.coxeter(n), mistake) != mahonian(n)
        or _bfs_variant(n, I.all_transpositions(n), mistake) != transposition_growth(n)
        or _bfs_variant(n, I.pancake(n), mistake) != scipy_growth(n, I.pancake(n))
    )
    assert caught


def test_two_layer_window_is_wrong_for_directed_sets():
    # The window of layers d and d-1 is exact only for inverse-closed sets;
    # the directed LX graph exposes the difference.
    n = 6
    expected = scipy_growth(n, I.lx(n), directed=True)
    assert _bfs_variant(n, I.lx(n), "only_previous_layer") != expected
    # for an inverse-closed set the window gives the exact answer
    assert _bfs_variant(n, I.lrx(n), "only_previous_layer") == scipy_growth(n, I.lrx(n))
