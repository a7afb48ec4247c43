"""ORACLE: plain CPU implementations of Cayley-graph growth (test infrastructure).

This package is test infrastructure. Only ``tests/``, ``__graft_entry__``
(``build()`` compiles it, ``smoke()`` checks the GPU against it) and the
CPU-baseline leg of ``bench.py`` may import or call it. The GPU path never
does, and the two share no code.

* ``bfs_set``  -- breadth-first search over a Python ``set`` of tuples.
* ``native``   -- the same search in plain C over an open-addressing hash set
                  of packed tuples (``bfs_hash.c``), fast enough for S_12.
* ``stats``    -- mean, mode, variance, skewness, kurtosis and moment-matched
                  Gaussian / Gumbel fits of a growth vector, from their
                  definitions (exact fractions for the moments).

Both follow the paper's definition of growth (section "Reminder on Cayley
graphs, diameters, growth"). Every function is pinned by tests against
closed forms, values printed in the paper and independent brute force.
"""
