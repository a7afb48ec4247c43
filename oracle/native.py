"""ORACLE (test infrastructure only): build and call the C hash-set BFS.

Only ``tests/``, ``__graft_entry__`` (building it, and the smoke check) and
the CPU-baseline leg of ``bench.py`` may use this module. See ``bfs_hash.c``
for what the C code computes and which passage of the paper it follows.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bfs_hash.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_handle = None


def build(force: bool = True) -> str:
    """Compile ``bfs_hash.c`` with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _lib():
    global _handle
    if _handle is None:
        if not os.path.exists(_LIB):
            build(force=True)
        h = ctypes.CDLL(_LIB)
        h.oracle_growth.restype = ctypes.c_int
        h.oracle_growth.argtypes = [
            ctypes.c_int,
            ctypes.c_void_p,
            ctypes.c_int,
            ctypes.c_void_p,
            ctypes.c_int,
            ctypes.c_uint64,
            ctypes.c_void_p,
            ctypes.POINTER(ctypes.c_int),
            ctypes.c_void_p,
            ctypes.c_uint64,
            ctypes.POINTER(ctypes.c_uint64),
        ]
        _handle = h
    return _handle


def growth(
    n: int,
    gens: Sequence[Sequence[int]],
    max_layers: int = 4096,
    max_frontier: int = 0,
    start: Optional[Sequence[int]] = None,
    with_states: bool = False,
) -> Tuple[List[int], int, Optional[np.ndarray]]:
    """Run the C oracle.

    Returns ``(sizes, status, states)``: the recorded layer sizes, the status
    (0 complete, 1 truncated) and, if requested, every visited state as rows
    of ``uint8[n]`` in discovery order, layer after layer.
    """
    g = np.ascontiguousarray(np.asarray(gens, dtype=np.uint8).reshape(-1, n))
    k = g.shape[0]
    st = None if start is None else np.ascontiguousarray(np.asarray(start, dtype=np.uint8))
    sizes = np.zeros(max_layers, dtype=np.uint64)
    nl = ctypes.c_int(0)
    nv = ctypes.c_uint64(0)
    states = None
    cap = 0
    if with_states:
        # a first pass counts the states, a second one fills them in
        rc = _lib().oracle_growth(
            n, g.ctypes.data, k, None if st is None else st.ctypes.data, max_layers,
            max_frontier, sizes.ctypes.data, ctypes.byref(nl), None, 0, ctypes.byref(nv),
        )
        if rc < 0:
            raise RuntimeError(f"oracle_growth failed with code {rc}")
        cap = int(nv.value)
        states = np.zeros((max(cap, 1), n), dtype=np.uint8)
    rc = _lib().oracle_growth(
        n, g.ctypes.data, k, None if st is None else st.ctypes.data, max_layers,
        max_frontier, sizes.ctypes.data, ctypes.byref(nl),
        None if states is None else states.ctypes.data, cap, ctypes.byref(nv),
    )
    if rc < 0:
        raise RuntimeError(f"oracle_growth failed with code {rc}")
    out = [int(x) for x in sizes[: nl.value]]
    if states is not None:
        states = states[:cap]
    return out, rc, states
