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


def test_pack_ascii_matches_pack_host_and_rejects_non_acgt():
    """paf_pack_ascii: the same planar words as paf_pack_host on the codes
    A=0, C=1, G=2, T=3 (either case), with per-pair lengths and word offsets;
    any other byte inside a sequence is PAF_ERR_ARG and nothing is written."""
    import numpy as np
    import paper_1910_03936_amd as paf

    lib = paf.load_library()
    rng = np.random.default_rng(11)
    n, stride = 9, 300
    lens = np.array([1, 31, 32, 33, 64, 65, 100, 250, 300], np.uint16)
    codes = rng.integers(0, 4, (n, stride)).astype(np.uint8)
    letters = np.frombuffer(b"ACGT", np.uint8)[codes]
    lower = rng.random((n, stride)) < 0.3
    text = np.where(lower, letters + 32, letters).astype(np.uint8)   # mixed case
    # past each length: bytes that are not bases, which must not be read
    for p in range(n):
        text[p, lens[p]:] = ord("N")
    words_per = [(int(m) + 31) // 32 for m in lens]
    offs = np.concatenate([[0], np.cumsum(words_per)[:-1]]).astype(np.uint64)
    total = int(sum(words_per))
    P = ctypes.c_void_p

    def call(fn, rows, out):
        return fn(rows.ctypes.data_as(P), stride, lens.ctypes.data_as(P), 0, offs.ctypes.data_as(P), 0, n,
                  out.ctypes.data_as(P), 3)

    want = np.zeros(total, np.uint64)
    assert call(lib.paf_pack_host, codes, want) == 0
    got = np.zeros(total, np.uint64)
    assert call(lib.paf_pack_ascii, text, got) == 0
    assert np.array_equal(got, want)
    # the binding's helper on equal-length strings: one row per string
    seqs = ["".join("ACGT"[c] for c in codes[p, :100]) for p in range(n)]
    w2 = paf.pack_ascii(seqs)
    ref = np.zeros(n * 4, np.uint64)
    assert lib.paf_pack_host(codes.ctypes.data_as(P), stride, None, 100, None, 4, n, ref.ctypes.data_as(P), 1) == 0
    assert np.array_equal(w2, ref)
    # rejection: N (and other bytes) inside a sequence, words untouched
    for bad_byte in (ord("N"), ord("n"), ord("U"), 0, ord("-"), 0xC1):
        bad = text.copy()
        bad[7, 123] = bad_byte
        out = np.full(total, 0xABCD, np.uint64)
        assert call(lib.paf_pack_ascii, bad, out) == 1
        assert b"not A, C, G or T" in lib.paf_last_error()
        assert np.all(out == 0xABCD)
    # a length beyond the row is a range error
    big = lens.copy()
    big[0] = stride + 1
    out = np.zeros(total + 16, np.uint64)
    assert lib.paf_pack_ascii(text.ctypes.data_as(P), stride, big.ctypes.data_as(P), 0, offs.ctypes.data_as(P), 0, n,
                              out.ctypes.data_as(P), 2) == 2
    import pytest
    with pytest.raises(paf.PafError):
        paf.pack_ascii(["ACGTN"])
