"""Readers for the paper fixtures in ``tests/golden`` and closed-form pins.

The closed forms below are the mathematics the paper states (each function
names the passage); they are independent of any BFS code.
"""

from __future__ import annotations

import math
import os
from typing import List, Tuple

from paper_2509_19162_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def max_diameter_table(directed: bool) -> List[Tuple[int, int, List[List[int]]]]:
    """Rows (n, printed diameter, generators in one-line notation)."""
    name = "max_diameter_directed.txt" if directed else "max_diameter_undirected.txt"
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            n_s, d_s, gens_s = [x.strip() for x in line.split("|")]
            n = int(n_s)
            gens = [I.parse_cycles(n, g) for g in gens_s.split(";")]
            rows.append((n, int(d_s), gens))
    return rows


def mahonian(n: int) -> List[int]:
    """Coefficients of prod_{i=1..n} (1 + q + ... + q^(i-1)): the number of
    permutations with m inversions (Coxeter row of the summary table: the
    word metric is the inversion count)."""
    poly = [1]
    for i in range(1, n + 1):
        nxt = [0] * (len(poly) + i - 1)
        for a, c in enumerate(poly):
            for b in range(i):
                nxt[a + b] += c
        poly = nxt
    return poly


def stirling1_unsigned(n: int) -> List[int]:
    """c(n, k) for k = 0..n by c(n+1, k) = n c(n, k) + c(n, k-1)."""
    row = [1]  # n = 0
    for m in range(n):
        nxt = [0] * (len(row) + 1)
        for k in range(len(nxt)):
            nxt[k] = (m * row[k] if k < len(row) else 0) + (row[k - 1] if k >= 1 else 0)
        row = nxt
    return row


def transposition_growth(n: int) -> List[int]:
    """gamma(m) = c(n, n - m), m = 0..n-1 (all transpositions: distance is
    n minus the number of cycles)."""
    c = stirling1_unsigned(n)
    return [c[n - m] for m in range(n)]


def reversal_sphere2(n: int) -> int:
    """|S_2| = (n^4 - 2n^3 - n^2 - 16n + 42)/6 for the reversal graph."""
    v = n ** 4 - 2 * n ** 3 - n ** 2 - 16 * n + 42
    assert v % 6 == 0
    return v // 6


def binary_coset_growth(n: int) -> List[int]:
    """C(m,k)^2 for n = 2m, C(m,k) C(m+1,k) for n = 2m+1, k = 0..m."""
    m = n // 2
    if n % 2 == 0:
        return [math.comb(m, k) ** 2 for k in range(m + 1)]
    return [math.comb(m, k) * math.comb(m + 1, k) for k in range(m + 1)]


def lx_diameter(n: int) -> int:
    v = 3 * n * n - 8 * n + (9 if n % 2 else 12)
    assert v % 4 == 0
    return v // 4
