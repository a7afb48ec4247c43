"""ORACLE (test infrastructure only): breadth-first growth over a Python set.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module. The GPU path never does, and this
module imports nothing from it.

It computes the growth of a Cayley (or Schreier) graph exactly as the paper
defines it (section "Reminder on Cayley graphs, diameters, growth",
definition of Growth): gamma(m) is the number of vertices at shortest-path
distance m from the start vertex. Edges join v and v.g for every generator
g; states are vectors in one-line notation, 0-based (section "Examples and
Tutorials"). The action is taken as a gather, t[i] = s[g[i]] (the paper does
not fix the convention; layer sizes do not depend on it).

The search keeps the full visited set, so it is also correct for generating
sets that are not closed under inverses.
"""

from __future__ import annotations

from typing import Iterable, List, Optional, Sequence, Tuple

State = Tuple[int, ...]


def apply_gather(state: Sequence[int], gen: Sequence[int]) -> State:
    """Neighbour of ``state`` under ``gen``: position i takes entry gen[i]."""
    return tuple(state[gen[i]] for i in range(len(gen)))


def bfs_layers(
    n: int,
    gens: Iterable[Sequence[int]],
    max_layers: Optional[int] = None,
    max_frontier: Optional[int] = None,
    start: Optional[Sequence[int]] = None,
) -> Tuple[List[List[State]], bool]:
    """Layers of the BFS from ``start`` (default: the identity 0..n-1).

    Returns ``(layers, complete)``. ``layers[m]`` lists the states at
    distance m in discovery order. ``complete`` is True when the search
    found an empty next layer, False when a stop rule ended it:
    ``max_layers`` caps the number of recorded layers, and the first layer
    larger than ``max_frontier`` is recorded but not expanded.
    """
    gens = [tuple(int(x) for x in g) for g in gens]
    for g in gens:
        if len(g) != n or sorted(g) != list(range(n)):
            raise ValueError(f"generator {g} is not a permutation of 0..{n - 1}")
    root: State = tuple(range(n)) if start is None else tuple(int(x) for x in start)
    if len(root) != n:
        raise ValueError("start vector has the wrong length")
    visited = {root}
    layers: List[List[State]] = [[root]]
    while True:
        if max_frontier is not None and len(layers[-1]) > max_frontier:
            return layers, False
        if max_layers is not None and len(layers) >= max_layers:
            return layers, False
        nxt: List[State] = []
        for s in layers[-1]:
            for g in gens:
                t = apply_gather(s, g)
                if t not in visited:
                    visited.add(t)
                    nxt.append(t)
        if not nxt:
            return layers, True
        layers.append(nxt)


def growth(
    n: int,
    gens: Iterable[Sequence[int]],
    max_layers: Optional[int] = None,
    max_frontier: Optional[int] = None,
    start: Optional[Sequence[int]] = None,
) -> List[int]:
    """Growth vector gamma(0), gamma(1), ... (layer sizes)."""
    layers, _ = bfs_layers(n, gens, max_layers, max_frontier, start)
    return [len(layer) for layer in layers]
