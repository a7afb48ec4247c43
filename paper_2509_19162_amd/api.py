"""Python binding of libcayleygrowth.so: argument marshalling only.

Every step of the growth computation runs in the library's HIP kernels;
this module converts Python/numpy arguments into the C structures and
raises on negative status codes. PyTorch is used only to hand the library a
stream (``stream=torch.cuda.current_stream()``) when the caller wants one.
"""

from __future__ import annotations

import atexit
import ctypes
import weakref
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import _native as N


class CGError(RuntimeError):
    def __init__(self, code: int, detail: str):
        self.code = code
        msg = N.lib().cg_strerror(code).decode()
        super().__init__(f"{msg} ({code}): {detail}" if detail else f"{msg} ({code})")


@dataclass
class GrowthResult:
    status: int
    sizes: List[int]
    states_expanded: int
    candidates: int
    device_ms: float
    t_submit: float = 0.0
    t_admit: float = 0.0
    t_done: float = 0.0
    kstats: Dict[str, Dict[str, float]] = field(default_factory=dict)
    layers: Optional[List[np.ndarray]] = None

    @property
    def complete(self) -> bool:
        return self.status == N.CG_OK

    @property
    def diameter(self) -> int:
        return len(self.sizes) - 1


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(getattr(stream, "cuda_stream"))  # torch.cuda.Stream


def _gens_array(n: int, gens: Sequence[Sequence[int]]) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(gens, dtype=np.uint8).reshape(-1, n))
    return a


def _ptr(a: Optional[np.ndarray], t=N.u8p):
    if a is None:
        return None
    return a.ctypes.data_as(t)


def _check(rc: int) -> int:
    if rc < 0:
        raise CGError(rc, N.lib().cg_last_error().decode())
    return rc


class _JobHolder:
    """Keeps the numpy buffers of a CgJob alive."""

    def __init__(self, n, gens, max_layers, max_frontier, flags, start, export_cap):
        self.n = n
        self.gens = _gens_array(n, gens)
        self.start = None if start is None else np.ascontiguousarray(np.asarray(start, dtype=np.uint8))
        if self.start is not None:
            flags |= N.CG_START_STATE
        self.export = None
        if export_cap:
            self.export = np.zeros((export_cap, n), dtype=np.uint8)
        self.sizes = np.zeros(max_layers, dtype=np.uint64)
        self.job = N.CgJob(
            n, _ptr(self.gens), self.gens.shape[0], max_layers, max_frontier or 0, flags,
            _ptr(self.start), _ptr(self.export), export_cap or 0,
        )
        self.res = N.CgResult()
        self.res.layer_sizes = self.sizes.ctypes.data_as(N.u64p)

    def result(self) -> GrowthResult:
        r = self.res
        sizes = [int(x) for x in self.sizes[: r.num_layers]] if r.status >= 0 else []
        ks = {}
        for i in range(r.n_kstats):
            k = r.kstats[i]
            ks[k.name.decode()] = {
                "launches": int(k.launches),
                "total_ms": float(k.total_ms),
                "alg_bytes": float(k.alg_bytes),
                "items": float(k.items),
            }
        layers = None
        if self.export is not None and r.status >= 0:
            layers = []
            off = 0
            for s in sizes:
                layers.append(self.export[off: off + s])
                off += s
        return GrowthResult(
            r.status, sizes, int(r.states_expanded), int(r.candidates), float(r.device_ms),
            float(r.t_submit), float(r.t_admit), float(r.t_done), ks, layers,
        )


def growth(n: int, gens: Sequence[Sequence[int]], max_layers: int = 256,
           max_frontier: Optional[int] = None) -> List[int]:
    """Growth (layer sizes) of the Cayley graph from the identity
    (``cg_growth``). Raises CGError on failure."""
    g = _gens_array(n, gens)
    sizes = np.zeros(max_layers, dtype=np.uint64)
    if max_frontier:
        return growth_ex(n, gens, max_layers=max_layers, max_frontier=max_frontier).sizes
    rc = _check(N.lib().cg_growth(n, _ptr(g), g.shape[0], max_layers, sizes.ctypes.data_as(N.u64p)))
    nz = np.nonzero(sizes)[0]
    last = int(nz[-1]) + 1 if len(nz) else 0
    del rc
    return [int(x) for x in sizes[:last]]


def growth_ex(n: int, gens: Sequence[Sequence[int]], max_layers: int = 256,
              max_frontier: Optional[int] = None, start: Optional[Sequence[int]] = None,
              keep_all_layers: bool = False, allow_directed: bool = False, profile: bool = False,
              export_layers: int = 0, stream=None, packed_sort: bool = False,
              bitmask: bool = False, small_job: bool = False, binary_state: bool = False) -> GrowthResult:
    """The full job interface (``cg_growth_ex``). ``bitmask`` selects the
    rank-space bitmap engine (n <= 14, sizes only); ``small_job`` runs the
    job inside one workgroup (n <= 10, sizes only); ``binary_state`` packs a
    0/1 ``start`` vector one bit per entry (implied for n > 16, up to 64).

    ``export_layers``: capacity (in states) of the layer-content export; the
    result's ``layers`` then lists each layer's states in increasing
    lexicographic order as ``uint8[count, n]`` arrays.
    """
    flags = 0
    if keep_all_layers:
        flags |= N.CG_KEEP_ALL_LAYERS
    if allow_directed:
        flags |= N.CG_ALLOW_DIRECTED
    if profile:
        flags |= N.CG_PROFILE
    if packed_sort:
        flags |= N.CG_PACKED_SORT
    if bitmask:
        flags |= N.CG_BITMASK
    if small_job:
        flags |= N.CG_SMALL_JOB
    if binary_state:
        flags |= N.CG_BINARY_STATE
    h = _JobHolder(n, gens, max_layers, max_frontier, flags, start, export_layers)
    _check(N.lib().cg_growth_ex(ctypes.byref(h.job), ctypes.byref(h.res), _stream_handle(stream)))
    return h.result()


class Engine:
    """A reusable engine (``cg_engine_*``): keeps its stream and device
    buffers between runs. ``run`` takes the arguments of ``growth_ex``."""

    def __init__(self, stream=None):
        self._e = N.lib().cg_engine_create(_stream_handle(stream))
        if not self._e:
            raise CGError(N.CG_E_DEVICE, N.lib().cg_last_error().decode())

    def run(self, n: int, gens, max_layers: int = 256, max_frontier: Optional[int] = None,
            start=None, keep_all_layers: bool = False, allow_directed: bool = False,
            profile: bool = False, export_layers: int = 0, packed_sort: bool = False,
            bitmask: bool = False, small_job: bool = False, binary_state: bool = False) -> GrowthResult:
        flags = (N.CG_KEEP_ALL_LAYERS if keep_all_layers else 0) | \
                (N.CG_ALLOW_DIRECTED if allow_directed else 0) | (N.CG_PROFILE if profile else 0) | \
                (N.CG_PACKED_SORT if packed_sort else 0) | (N.CG_BITMASK if bitmask else 0) | \
                (N.CG_SMALL_JOB if small_job else 0) | (N.CG_BINARY_STATE if binary_state else 0)
        h = _JobHolder(n, gens, max_layers, max_frontier, flags, start, export_layers)
        _check(N.lib().cg_engine_run(self._e, ctypes.byref(h.job), ctypes.byref(h.res)))
        return h.result()

    def close(self):
        if self._e:
            N.lib().cg_engine_destroy(self._e)
            self._e = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _struct_dtype(ctype) -> np.dtype:
    """A numpy dtype with the byte layout of a ctypes structure (scalar and
    pointer fields by name; other fields as raw bytes)."""
    names, formats, offsets = [], [], []
    for name, t in ctype._fields_:
        f = getattr(ctype, name)
        if t in (ctypes.c_int, ctypes.c_uint32):
            fmt = np.int32 if t is ctypes.c_int else np.uint32
        elif t in (ctypes.c_uint64,) or t is N.u8p or t is N.u64p or t is ctypes.c_void_p:
            fmt = np.uint64
        elif t is ctypes.c_double:
            fmt = np.float64
        else:
            fmt = np.dtype((np.void, f.size))
        names.append(name)
        formats.append(fmt)
        offsets.append(f.offset)
    return np.dtype({"names": names, "formats": formats, "offsets": offsets, "itemsize": ctypes.sizeof(ctype)})


def _batch_arrays(jobs, max_layers: int, flags: int):
    """Job and result arrays of a batch in the C layouts, with the
    generators and layer sizes in two contiguous buffers."""
    m = len(jobs)
    ns = np.fromiter((j[0] for j in jobs), dtype=np.int32, count=m)
    g_arrays = [np.asarray(j[1], dtype=np.uint8).reshape(-1, int(j[0])) for j in jobs]
    rows = np.fromiter((a.shape[0] for a in g_arrays), dtype=np.int32, count=m)
    gens = np.ascontiguousarray(np.concatenate([a.ravel() for a in g_arrays])) if m else np.zeros(1, np.uint8)
    goff = np.zeros(m, dtype=np.uint64)
    if m > 1:
        goff[1:] = np.cumsum((rows.astype(np.uint64) * ns.astype(np.uint64))[:-1])
    mf = np.fromiter(((j[2] or 0) if len(j) > 2 else 0 for j in jobs), dtype=np.uint64, count=m)
    ml = np.fromiter(((j[3] or max_layers) if len(j) > 3 else max_layers for j in jobs), dtype=np.int32, count=m)
    soff = np.zeros(m, dtype=np.uint64)
    if m > 1:
        soff[1:] = np.cumsum(ml[:-1].astype(np.uint64))
    sizes = np.zeros(max(int(ml.sum()), 1), dtype=np.uint64)
    ja = np.zeros(m, dtype=_struct_dtype(N.CgJob))
    ja["n"] = ns
    ja["gens"] = np.uint64(gens.ctypes.data) + goff
    ja["n_gens"] = rows
    ja["max_layers"] = ml
    ja["max_frontier"] = mf
    ja["flags"] = flags
    ra = np.zeros(m, dtype=_struct_dtype(N.CgResult))
    ra["layer_sizes"] = np.uint64(sizes.ctypes.data) + soff * np.uint64(8)
    return ja, ra, gens, sizes, soff


def _batch_results(ra, sizes, soff) -> List[GrowthResult]:
    out = []
    status = ra["status"].tolist()
    nl = ra["num_layers"].tolist()
    se = ra["states_expanded"].tolist()
    ca = ra["candidates"].tolist()
    dm = ra["device_ms"].tolist()
    ts, tad, td = ra["t_submit"].tolist(), ra["t_admit"].tolist(), ra["t_done"].tolist()
    so = soff.tolist()
    for i in range(len(status)):
        sz = sizes[so[i]: so[i] + nl[i]].tolist() if status[i] >= 0 else []
        out.append(GrowthResult(status[i], sz, se[i], ca[i], dm[i], ts[i], tad[i], td[i], {}, None))
    return out


def growth_batch(jobs, max_layers: int = 256, max_active: int = 0, budget_bytes: int = 0,
                 tune: bool = False, stream=None, allow_directed: bool = False) -> List[GrowthResult]:
    """Many independent jobs in shared super-steps (``cg_growth_batch``).

    ``jobs``: a list of ``(n, gens)``, ``(n, gens, max_frontier)`` or
    ``(n, gens, max_frontier, max_layers)``. Per-job failures (a bad
    generator row) show up as a negative ``status`` in that job's result.
    """
    ja, ra, gens, sizes, soff = _batch_arrays(jobs, max_layers, N.CG_ALLOW_DIRECTED if allow_directed else 0)
    opts = N.CgBatchOpts(_stream_handle(stream), max_active, budget_bytes, 1 if tune else 0)
    _check(N.lib().cg_growth_batch(len(jobs), ja.ctypes.data_as(ctypes.POINTER(N.CgJob)),
                                   ra.ctypes.data_as(ctypes.POINTER(N.CgResult)), ctypes.byref(opts)))
    return _batch_results(ra, sizes, soff)


def batch_info() -> Dict[str, float]:
    """What ``cg_growth_batch`` keeps on the current device (``cg_batch_info``):
    calls, launch graphs built and launched (replays = launches - builds),
    autotuned classes, the tuned heavy-job split, entries read from the
    tuning file."""
    st = N.CgBatchInfo()
    _check(N.lib().cg_batch_info(ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in N.CgBatchInfo._fields_}


def growth_batch_noalloc(jobs, max_layers: int = 256, stream=None,
                         allow_directed: bool = False) -> List[GrowthResult]:
    """``cg_growth_batch_noalloc``: the jobs of ``growth_batch`` (each with
    n <= 10) run without any device allocation, on the library's static
    device array. Same job tuple forms as ``growth_batch``."""
    ja, ra, gens, sizes, soff = _batch_arrays(jobs, max_layers, N.CG_ALLOW_DIRECTED if allow_directed else 0)
    _check(N.lib().cg_growth_batch_noalloc(len(jobs), ja.ctypes.data_as(ctypes.POINTER(N.CgJob)),
                                           ra.ctypes.data_as(ctypes.POINTER(N.CgResult)), _stream_handle(stream)))
    return _batch_results(ra, sizes, soff)


def release_cached_memory() -> None:
    """Frees the buffers that batches keep between calls, then returns the
    library's device arena to HIP (hipFree) when no buffer uses it
    (``cg_release_cached_memory``)."""
    N.lib().cg_release_cached_memory()


def memory_stats(reset_peak: bool = False) -> Dict[str, int]:
    """Bytes the library's device buffers hold now and at most since the
    last reset, and the arenas' reserved size (``cg_memory_stats``)."""
    st = N.CgMemoryStats()
    _check(N.lib().cg_memory_stats(ctypes.byref(st), 1 if reset_peak else 0))
    return {f: int(getattr(st, f)) for f, _ in N.CgMemoryStats._fields_}


_WORKSPACE = None  # keeps the caller's tensor alive while the library uses it


def set_workspace(tensor) -> None:
    """Let the library carve its device buffers out of ``tensor`` (a CUDA
    tensor, e.g. ``torch.empty(nbytes, dtype=torch.uint8, device="cuda")``)
    (``cg_set_workspace``); ``None`` returns to library-reserved memory.
    Close engines and queues first (their buffers live in the old arena)."""
    global _WORKSPACE
    if tensor is None:
        _check(N.lib().cg_set_workspace(None, 0))
        _WORKSPACE = None
        return
    if not tensor.is_cuda or not tensor.is_contiguous():
        raise ValueError("workspace must be a contiguous device tensor")
    nbytes = tensor.numel() * tensor.element_size()
    _check(N.lib().cg_set_workspace(ctypes.c_void_p(tensor.data_ptr()), nbytes))
    _WORKSPACE = tensor


def growth_stats(sizes: Sequence[int]) -> Dict[str, float]:
    """Statistics of a growth vector (``cg_growth_stats``): mean, mode,
    variance, skewness, excess kurtosis, moment-matched Gaussian and Gumbel
    fits and their total-variation distances."""
    a = np.ascontiguousarray(np.asarray(list(sizes), dtype=np.uint64))
    if a.size == 0:
        raise CGError(N.CG_E_INVAL, "empty growth vector")
    st = N.CgGrowthStats()
    _check(N.lib().cg_growth_stats(a.ctypes.data_as(N.u64p), int(a.size), ctypes.byref(st)))
    out = {name: getattr(st, name) for name, _ in N.CgGrowthStats._fields_}
    out["gumbel_min"] = bool(out["gumbel_min"])
    out["best_fit"] = "gumbel" if out["best_fit"] else "gaussian"
    return out


_LIVE_QUEUES: "weakref.WeakSet[GrowthQueue]" = weakref.WeakSet()


@atexit.register
def _close_live_queues():
    # a queue's engine threads must stop before the interpreter and the HIP
    # runtime shut down, even if the caller never closed it
    for q in list(_LIVE_QUEUES):
        q.close()


class GrowthQueue:
    """Request queue with continuous batching (``cg_queue_*``). Use as a
    context manager or call ``close()``; open queues are closed at exit."""

    def __init__(self, budget_bytes: int = 0, max_active: int = 0, max_queued: int = 0,
                 large_lanes: int = 0, device: int = -1, stream=None):
        opts = N.CgQueueOpts(budget_bytes, max_active, max_queued, large_lanes, device, _stream_handle(stream))
        self._q = N.lib().cg_queue_create(ctypes.byref(opts))
        if not self._q:
            raise CGError(N.CG_E_DEVICE, N.lib().cg_last_error().decode())
        self._jobs: Dict[int, _JobHolder] = {}
        _LIVE_QUEUES.add(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, n: int, gens, max_layers: int = 256, max_frontier: Optional[int] = None,
               start=None, allow_directed: bool = False) -> int:
        h = _JobHolder(n, gens, max_layers, max_frontier, N.CG_ALLOW_DIRECTED if allow_directed else 0, start, 0)
        t = ctypes.c_uint64(0)
        _check(N.lib().cg_queue_submit(self._q, ctypes.byref(h.job), ctypes.byref(h.res), ctypes.byref(t)))
        self._jobs[int(t.value)] = h
        return int(t.value)

    def poll(self, ticket: int) -> int:
        return N.lib().cg_queue_poll(self._q, ticket)

    def wait(self, ticket: int, timeout_s: Optional[float] = None) -> GrowthResult:
        us = -1 if timeout_s is None else int(timeout_s * 1e6)
        rc = N.lib().cg_queue_wait(self._q, ticket, us)
        if rc == N.CG_E_TIMEOUT:
            raise TimeoutError(f"ticket {ticket} still running")
        h = self._jobs.pop(ticket)
        if rc < 0:
            raise CGError(rc, N.lib().cg_last_error().decode())
        return h.result()

    def cancel(self, ticket: int) -> int:
        return N.lib().cg_queue_cancel(self._q, ticket)

    def stats(self) -> Dict[str, int]:
        """Admission accounting (``cg_queue_stats``): budget, charged and
        held device bytes with their peaks, running and queued jobs, and
        completed / cancelled / failed counts."""
        st = N.CgQueueStats()
        _check(N.lib().cg_queue_stats(self._q, ctypes.byref(st)))
        return {name: int(getattr(st, name)) for name, _ in N.CgQueueStats._fields_}

    def close(self):
        if self._q:
            N.lib().cg_queue_destroy(self._q)
            self._q = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
