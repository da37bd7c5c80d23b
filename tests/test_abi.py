"""The C-ABI library loads and exports every entry point include/paf.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

from tests.conftest import ROOT


def _declared():
    with open(os.path.join(ROOT, "include", "paf.h")) as f:
        src = f.read()
    return sorted(set(re.findall(r"^\s*(?:paf_status|const char\*)\s+(paf_\w+)\s*\(", src, re.M)))


def test_header_declares_entry_points():
    names = _declared()
    assert "paf_filter" in names and "paf_create" in names and len(names) >= 15


def test_library_exports_every_declared_symbol():
    import paper_1910_03936_amd as paf

    assert os.path.exists(paf.LIB_PATH), "build the library first (__graft_entry__.build())"
    lib = ctypes.CDLL(paf.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_declared()) == set(paf.EXPORTS)


def test_binding_loads_and_reports_errors_without_gpu():
    import paper_1910_03936_amd as paf

    lib = paf.load_library()
    # A call with a NULL context is rejected on the host before any device work.
    st = lib.paf_check(None, None)
    assert st == 1
    assert b"ctx" in lib.paf_last_error()


def test_pack_host_layout():
    """paf_pack_host: planar two-bit words (host-only entry point)."""
    import numpy as np
    import paper_1910_03936_amd as paf

    lib = paf.load_library()
    rng = np.random.default_rng(0)
    n, m = 5, 70
    codes = rng.integers(0, 4, (n, 80)).astype(np.uint8)
    words = np.zeros(n * 3, np.uint64)
    st = lib.paf_pack_host(codes.ctypes.data_as(ctypes.c_void_p), 80, None, m, None, 3, n,
                           words.ctypes.data_as(ctypes.c_void_p), 2)
    assert st == 0
    for p in range(n):
        for k in range(3):
            w = int(words[p * 3 + k])
            for j in range(32):
                i = 32 * k + j
                c = int(codes[p, i]) if i < m else 0
                assert (w >> j) & 1 == c & 1
                assert (w >> (32 + j)) & 1 == c >> 1
    bad = codes.copy()
    bad[2, 5] = 7
    st = lib.paf_pack_host(bad.ctypes.data_as(ctypes.c_void_p), 80, None, m, None, 3, n,
                           words.ctypes.data_as(ctypes.c_void_p), 2)
    assert st == 2
