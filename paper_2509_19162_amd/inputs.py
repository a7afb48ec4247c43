"""Seeded synthetic inputs: generator families, cycle notation, random sets.

This module only builds inputs (generator rows in one-line notation). It
holds none of the growth computation, so both the GPU path's tests and the
CPU oracle may be fed from it.

Conventions (paper, section "Examples and Tutorials" and the definitions of
the named generators in section "Sheveleva2 and Koltsov3involutions"):
a generator is a permutation of 0..n-1 in one-line notation, 0-based, and it
acts on a state by gather, t[i] = s[g[i]].
"""

from __future__ import annotations

import itertools
import math
from typing import List, Optional, Sequence

import numpy as np

#: Seed of every synthetic workload (the arXiv number of the paper).
SEED = 19162

Perm = List[int]


def identity(n: int) -> Perm:
    return list(range(n))


def transposition(n: int, i: int, j: int) -> Perm:
    g = identity(n)
    g[i], g[j] = g[j], g[i]
    return g


def inverse(g: Sequence[int]) -> Perm:
    inv = [0] * len(g)
    for i, x in enumerate(g):
        inv[x] = i
    return inv


def compose(a: Sequence[int], b: Sequence[int]) -> Perm:
    """One-line product: position i takes a[b[i]] (apply b's gather to a)."""
    return [a[b[i]] for i in range(len(b))]


# --- named families (table "Summary of properties of Cayley graphs") -----

def coxeter(n: int) -> List[Perm]:
    """Adjacent transpositions (i, i+1), i = 0..n-2 (bubble-sort graph)."""
    return [transposition(n, i, i + 1) for i in range(n - 1)]


def cyclic_coxeter(n: int) -> List[Perm]:
    """Coxeter generators plus the wrap-around transposition (0, n-1)."""
    gens = coxeter(n)
    if n > 2:
        gens.append(transposition(n, 0, n - 1))
    return gens


def all_transpositions(n: int) -> List[Perm]:
    return [transposition(n, i, j) for i in range(n) for j in range(i + 1, n)]


def star(n: int) -> List[Perm]:
    """Star transpositions (0, i), i = 1..n-1."""
    return [transposition(n, 0, i) for i in range(1, n)]


def pancake(n: int) -> List[Perm]:
    """Prefix reversals of length 2..n."""
    return [list(range(l - 1, -1, -1)) + list(range(l, n)) for l in range(2, n + 1)]


def left_shift(n: int) -> Perm:
    """L: t[i] = s[(i + 1) mod n]."""
    return [(i + 1) % n for i in range(n)]


def lrx(n: int) -> List[Perm]:
    """L (left cyclic shift), R = L^-1 and X = swap of positions 0 and 1."""
    L = left_shift(n)
    return [L, inverse(L), transposition(n, 0, 1)]


def lx(n: int) -> List[Perm]:
    """L and X only: not closed under inverses (directed graph)."""
    return [left_shift(n), transposition(n, 0, 1)]


def reversals(n: int) -> List[Perm]:
    """All segment reversals r_{i,j}, 0 <= i < j <= n-1."""
    out = []
    for i in range(n):
        for j in range(i + 1, n):
            out.append(list(range(i)) + list(range(j, i - 1, -1)) + list(range(j + 1, n)))
    return out


def transposons(n: int) -> List[Perm]:
    """Block transpositions: exchange the adjacent blocks [i, j) and [j, k)."""
    out = []
    for i in range(n):
        for j in range(i + 1, n):
            for k in range(j + 1, n + 1):
                out.append(list(range(i)) + list(range(j, k)) + list(range(i, j)) + list(range(k, n)))
    return out


def three_cycles(n: int) -> List[Perm]:
    """All 3-cycles (both orientations of every 3-subset)."""
    out = []
    for a, b, c in itertools.combinations(range(n), 3):
        for x, y, z in ((a, b, c), (a, c, b)):
            g = identity(n)
            # cycle x -> y -> z -> x on values: one-line image sends position x to y
            g[x], g[y], g[z] = y, z, x
            out.append(g)
    return out


# --- cycle notation (tables of largest diameters) --------------------------

def parse_cycles(n: int, text: str) -> Perm:
    """Parse a product of disjoint cycles such as ``(14)(26)(35)`` or
    ``(1,11,9,10)(04)`` into one-line notation.

    Entries are 0-based. A cycle without commas lists one digit per
    character; a cycle with commas lists comma-separated integers. The cycle
    (a b c) sends a to b, b to c and c to a; the one-line image at position a
    is b. (Growth does not depend on this choice, since a permutation and its
    inverse generate the same graph up to the inversion map.)
    """
    g = identity(n)
    used = set()
    for body in text.replace(" ", "").split(")"):
        if not body:
            continue
        if not body.startswith("("):
            raise ValueError(f"bad cycle text {text!r}")
        body = body[1:]
        items = [int(x) for x in body.split(",")] if "," in body else [int(c) for c in body]
        for x in items:
            if x < 0 or x >= n or x in used:
                raise ValueError(f"bad cycle entry {x} in {text!r} for n={n}")
            used.add(x)
        for a, b in zip(items, items[1:] + items[:1]):
            g[a] = b
    return g


# --- seeded random sets -----------------------------------------------------

def rng_for(job_id: int, seed: int = SEED) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([seed, job_id]))


def random_perms_with_inverses(n: int, m: int, rng: np.random.Generator) -> List[Perm]:
    """m uniform permutations of S_n (Fisher-Yates) followed by their inverses."""
    perms = [[int(x) for x in rng.permutation(n)] for _ in range(m)]
    return perms + [inverse(p) for p in perms]


def random_involution(n: int, rng: np.random.Generator) -> Perm:
    """A random involution with at least one 2-cycle.

    The number c of 2-cycles is drawn with probability proportional to the
    number of involutions with c 2-cycles, n!/(c! 2^c (n-2c)!); then a
    uniform 2c-subset is paired uniformly.
    """
    cs = list(range(1, n // 2 + 1))
    w = np.array([math.factorial(n) // (math.factorial(c) * 2 ** c * math.factorial(n - 2 * c)) for c in cs],
                 dtype=np.float64)
    c = int(rng.choice(cs, p=w / w.sum()))
    pts = [int(x) for x in rng.permutation(n)[: 2 * c]]
    g = identity(n)
    for a, b in zip(pts[0::2], pts[1::2]):
        g[a], g[b] = b, a
    return g


def random_involutions(n: int, m: int, rng: np.random.Generator) -> List[Perm]:
    return [random_involution(n, rng) for _ in range(m)]


def binary_central_state(n: int) -> List[int]:
    """Sorted binary vector with floor(n/2) zeros (binary coset start)."""
    z = n // 2
    return [0] * z + [1] * (n - z)


# --- the benchmark workloads -------------------------------------------------

def batch_jobs(n_jobs: int = 4096, seed: int = SEED):
    """Batched workload: n ~ U{7..10}, m ~ U{2,3,4} uniform random
    permutations plus their inverses, full growth for every job."""
    jobs = []
    for j in range(n_jobs):
        r = rng_for(j, seed)
        n = int(r.integers(7, 11))
        m = int(r.integers(2, 5))
        jobs.append((n, random_perms_with_inverses(n, m, r)))
    return jobs


SERVING_FAMILIES = ("all_transpositions", "star", "pancake", "lrx", "random_involutions")


def serving_request(req_id: int, seed: int = SEED, n_lo: int = 6, n_hi: int = 13):
    """One request of the serving workload: n ~ U{n_lo..n_hi} and a family
    drawn uniformly from SERVING_FAMILIES (2-4 random involutions for the
    last one)."""
    r = rng_for(1_000_000 + req_id, seed)
    n = int(r.integers(n_lo, n_hi + 1))
    fam = SERVING_FAMILIES[int(r.integers(0, len(SERVING_FAMILIES)))]
    if fam == "random_involutions":
        gens = random_involutions(n, int(r.integers(2, 5)), r)
    else:
        gens = FAMILIES[fam](n)
    return n, fam, gens


FAMILIES = {
    "coxeter": coxeter,
    "cyclic_coxeter": cyclic_coxeter,
    "all_transpositions": all_transpositions,
    "star": star,
    "pancake": pancake,
    "lrx": lrx,
    "lx": lx,
    "reversals": reversals,
    "transposons": transposons,
    "three_cycles": three_cycles,
}


def family(name: str, n: int) -> List[Perm]:
    return FAMILIES[name](n)


def as_array(gens: Sequence[Sequence[int]], n: Optional[int] = None) -> np.ndarray:
    a = np.asarray(gens, dtype=np.uint8)
    if n is not None:
        a = a.reshape(-1, n)
    return np.ascontiguousarray(a)
