"""CPU checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad arguments before touching the device."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2509_19162_amd import _native as N
from paper_2509_19162_amd import api
from paper_2509_19162_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in ("cayleygrowth.h", "cayleygrowth_testing.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(cg_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    lib = N.lib()
    names = declared_functions()
    assert {"cg_growth", "cg_growth_ex", "cg_growth_batch", "cg_queue_create"} <= names
    for name in names:
        assert hasattr(lib, name), name
    # the ctypes table covers exactly the declared functions
    assert {s[0] for s in N.SIGNATURES} == names


def test_struct_layout_matches_header():
    # offsets fixed by the C declaration order on x86-64
    assert ctypes.sizeof(N.CgJob) == 64
    assert N.CgResult.layer_sizes.offset == 8
    assert ctypes.sizeof(N.CgKstat) == 64


def test_strerror():
    lib = N.lib()
    assert lib.cg_strerror(0) == b"complete"
    assert lib.cg_strerror(-4) == b"unsupported generating set"


@pytest.mark.parametrize(
    "n,gens,why",
    [
        (0, [[0]], "n"),
        (17, [list(range(17))], "n"),
        (4, [[0, 1, 2, 2]], "not a permutation"),
        (4, [[0, 1, 2, 4]], "not a permutation"),
    ],
)
def test_invalid_jobs_are_rejected(n, gens, why):
    g = np.asarray(gens, dtype=np.uint8)
    sizes = np.zeros(8, dtype=np.uint64)
    rc = N.lib().cg_growth(n, g.ctypes.data_as(N.u8p), g.shape[0], 8, sizes.ctypes.data_as(N.u64p))
    assert rc == N.CG_E_INVAL
    assert why in N.lib().cg_last_error().decode()


def test_zero_generators_and_bad_layers_rejected():
    g = np.asarray([[1, 0]], dtype=np.uint8)
    sizes = np.zeros(8, dtype=np.uint64)
    lib = N.lib()
    assert lib.cg_growth(2, g.ctypes.data_as(N.u8p), 0, 8, sizes.ctypes.data_as(N.u64p)) == N.CG_E_INVAL
    assert lib.cg_growth(2, g.ctypes.data_as(N.u8p), 1, 0, sizes.ctypes.data_as(N.u64p)) == N.CG_E_INVAL
    assert lib.cg_growth(2, g.ctypes.data_as(N.u8p), 1, 8, None) == N.CG_E_INVAL


def test_directed_set_needs_flag():
    with pytest.raises(api.CGError) as e:
        api.growth(6, I.lx(6))
    assert e.value.code == N.CG_E_UNSUPPORTED


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(N, "_lib", None)
    monkeypatch.setattr(N, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(N.NativeLibraryMissing):
        N.lib()


def test_noalloc_batch_rejects_sizes_beyond_its_limits():
    """cg_growth_batch_noalloc checks its stated limits on the host, before
    any device call."""
    lib = N.lib()
    with pytest.raises(api.CGError) as e:
        api.growth_batch_noalloc([(5, I.coxeter(5))] * 4097)
    assert e.value.code == N.CG_E_INVAL and "4096" in str(e.value)
    with pytest.raises(api.CGError) as e:
        api.growth_batch_noalloc([(5, I.coxeter(5)), (11, I.coxeter(11))])
    assert e.value.code == N.CG_E_INVAL and "n <= 10" in str(e.value)
    with pytest.raises(api.CGError) as e:
        api.growth_batch_noalloc([(8, I.all_transpositions(8))] * 4096)  # 28 generators each
    assert e.value.code == N.CG_E_INVAL and "32768" in str(e.value)
    with pytest.raises(api.CGError) as e:
        api.growth_batch_noalloc([(10, [I.transposition(10, 0, 1)])] * 4096, max_layers=1024)
    assert e.value.code == N.CG_E_INVAL and "2^21" in str(e.value)
    # a directed set without the flag fails its own job (nothing to launch)
    res = api.growth_batch_noalloc([(6, I.lx(6))])
    assert res[0].status == N.CG_E_UNSUPPORTED
    assert lib.cg_growth_batch_noalloc(-1, None, None, None) == N.CG_E_INVAL


def test_binary_state_jobs_are_validated():
    """Binary states (one bit per entry) need a 0/1 start vector; n runs to
    64; they take the sort path only. All rejected before any device call."""
    lib = N.lib()
    sizes = np.zeros(8, dtype=np.uint64)

    def run(n, start, flags, gens=None):
        g = np.ascontiguousarray(np.asarray(gens if gens is not None else [I.coxeter(n)[0]], dtype=np.uint8))
        st = None if start is None else np.ascontiguousarray(np.asarray(start, dtype=np.uint8))
        job = N.CgJob(n, g.ctypes.data_as(N.u8p), g.shape[0], 8, 0, flags,
                      None if st is None else st.ctypes.data_as(N.u8p), None, 0)
        res = N.CgResult()
        res.layer_sizes = sizes.ctypes.data_as(N.u64p)
        return lib.cg_growth_ex(ctypes.byref(job), ctypes.byref(res), None), lib.cg_last_error().decode()

    half = lambda n: [0] * (n // 2) + [1] * (n - n // 2)  # noqa: E731
    rc, msg = run(65, half(65), N.CG_START_STATE, gens=[list(range(65))])
    assert rc == N.CG_E_INVAL and "1..64" in msg
    rc, msg = run(20, None, 0)
    assert rc == N.CG_E_INVAL and "start" in msg
    rc, msg = run(20, [2] + half(19), N.CG_START_STATE)
    assert rc == N.CG_E_INVAL and "0/1" in msg
    rc, msg = run(8, None, N.CG_BINARY_STATE)
    assert rc == N.CG_E_INVAL and "start" in msg
    rc, msg = run(20, half(20), N.CG_START_STATE | N.CG_BITMASK)
    assert rc == N.CG_E_INVAL and "sort path" in msg
    rc, msg = run(20, half(20), N.CG_START_STATE | N.CG_SMALL_JOB)
    assert rc == N.CG_E_INVAL and "sort path" in msg


def test_sort_hooks_validate_before_touching_the_device():
    """The testing ABI's sorts reject bad bit ranges and null buffers before
    any device call (so this runs without a GPU)."""
    lib = N.lib()
    for kb in (0, 65, -3):
        assert lib.cg_test_sort_below(None, None, 0, kb, None) == N.CG_E_INVAL
    assert lib.cg_test_sort_below(None, None, 5, 45, None) == N.CG_E_INVAL
    assert lib.cg_test_sort(None, None, 0, 8, 4, None) == N.CG_E_INVAL
    assert lib.cg_test_sort(None, None, 0, 0, 65, None) == N.CG_E_INVAL
    assert lib.cg_test_sort32(None, None, 0, 0, 33, None) == N.CG_E_INVAL
