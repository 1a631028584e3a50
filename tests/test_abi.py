"""CPU-side checks of the C ABI: the library loads without a GPU and exports
every function that include/bisim.h declares."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "bisim.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b([a-z_][a-z0-9_]*)\s*\(", txt, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "defined")))


def test_header_declares_expected():
    from paper_2105_11788_amd import bisim
    assert set(bisim.EXPORTS) <= set(header_functions())


def test_library_exports_every_declared_symbol():
    from paper_2105_11788_amd import bisim
    if not os.path.exists(bisim.LIB_PATH):
        pytest.skip("libbisim.so not built")
    L = bisim.load_library()
    for name in header_functions():
        assert hasattr(L, name), name


def test_last_error_without_gpu():
    from paper_2105_11788_amd import bisim
    if not os.path.exists(bisim.LIB_PATH):
        pytest.skip("libbisim.so not built")
    L = bisim.load_library()
    assert isinstance(L.bisim_last_error(), bytes)
    # argument validation happens before any device call
    import ctypes
    h = ctypes.c_void_p()
    assert L.lts_load(None, None, None, -1, 0, 1, None, None, ctypes.byref(h)) == bisim.E_INVALID
    assert b"n >= 0" in L.bisim_last_error()
    assert L.lts_load(None, None, None, 1, 0, 0, None, None, ctypes.byref(h)) == bisim.E_INVALID
    assert L.bisim_set_option(None, 1, 0) == bisim.E_INVALID
    # the query calls reject a NULL handle the same way
    v = ctypes.c_int32(0)
    L.bisim_get_preprocess_method.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert L.bisim_get_preprocess_method(None, ctypes.byref(v)) == bisim.E_INVALID
    L.bisim_get_run_config.argtypes = [ctypes.c_void_p] * 3
    assert L.bisim_get_run_config(None, ctypes.byref(v), ctypes.byref(v)) == bisim.E_INVALID


def test_noalloc_rejects_oversize_before_device_work():
    """The allocation-free entry point checks its static region's bound from
    n, m and K before any device call (so this runs without a GPU)."""
    from paper_2105_11788_amd import bisim
    if not os.path.exists(bisim.LIB_PATH):
        pytest.skip("libbisim.so not built")
    import ctypes
    L = bisim.load_library()
    st = bisim.bisim_stats()
    fake = ctypes.c_void_p(256)  # never dereferenced: the size check comes first
    n = bisim.NOALLOC_SCRATCH_BYTES // 64  # ~100 bytes per state needed: too large
    rc = L.coarsest_partition_noalloc(None, None, None, n, 0, 1, None, fake, ctypes.byref(st), None)
    assert rc == bisim.E_UNSUPPORTED
    assert b"static region" in L.bisim_last_error()
    rc = L.coarsest_partition_noalloc(None, None, None, 10, 0, 1, None, None, ctypes.byref(st), None)
    assert rc == bisim.E_INVALID  # NULL output
