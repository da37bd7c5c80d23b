"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct implementations of what the GPU path computes
(SneakySnake on the unweighted and weighted maze, on a column-partitioned maze
and in its hardware form, GateKeeper, Shouji, MAGNET, banded and full
Levenshtein distance, the cost-model features, and the cost-model MLP in
float64).  Only the tests, the package's smoke check and the benchmark's CPU
baseline leg may import this package; the product path never does.  It shares
no code with the GPU library: the C part (oracle.c) is compiled by gcc into its
own shared object, and the MLP reference (mlp.py) is numpy.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SNEAKYSNAKE, GATEKEEPER, SHOUJI = 1, 2, 4


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2 C, OpenMP only across pairs)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P, I = ctypes.c_void_p, ctypes.c_int
        lib.or_sneakysnake.argtypes = [P, P, I, I, P, P, I, P]
        lib.or_sneakysnake_weighted.argtypes = [P, P, I, I, P]
        lib.or_sneakysnake_t.argtypes = [P, P, I, I, I, P]
        lib.or_magnet.argtypes = [P, P, I, I, P, P, P]
        lib.or_sneakysnake_fpga.argtypes = [P, P, I, I, I, I, P]
        lib.or_sneakysnake_fpga_batch.argtypes = [P, P, ctypes.c_uint32, P, P, ctypes.c_uint64, I, I, P, P, I]
        lib.or_sneakysnake_fpga_batch.restype = None
        lib.or_magnet_batch.argtypes = [P, P, ctypes.c_uint32, P, P, ctypes.c_uint64, P, P, I]
        lib.or_magnet_batch.restype = None
        lib.or_sneakysnake_t_batch.argtypes = [P, P, ctypes.c_uint32, P, P, ctypes.c_uint64, I, P, P, I]
        lib.or_sneakysnake_t_batch.restype = None
        lib.or_gatekeeper.argtypes = [P, P, I, I, P]
        lib.or_shouji.argtypes = [P, P, I, I, P, P]
        lib.or_banded_levenshtein.argtypes = [P, P, I, I]
        lib.or_levenshtein.argtypes = [P, I, P, I]
        lib.or_hamming.argtypes = [P, P, I]
        lib.or_features.argtypes = [P, P, I, I, P]
        lib.or_amend.argtypes = [P, P, I]
        lib.or_amend.restype = None
        lib.or_filter_batch.argtypes = [P, P, ctypes.c_uint32, P, P, ctypes.c_uint64,
                                        ctypes.c_uint32, P, P, P, P, P, P, I]
        lib.or_filter_batch.restype = None
        lib.or_banded_batch.argtypes = [P, P, ctypes.c_uint32, P, P, ctypes.c_uint64, P, I]
        lib.or_banded_batch.restype = None
        lib.or_features_batch.argtypes = [P, P, ctypes.c_uint32, P, P, ctypes.c_uint64, P, I]
        lib.or_features_batch.restype = None
        _lib = lib
    return _lib


def _u8(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint8))


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def sneakysnake(read, ref, E, with_pipes=False):
    """(accept, count[, pipes]) for one pair; pipes = [(start col, diagonal, depth)]."""
    lib = _load()
    rd, rf = _u8(read), _u8(ref)
    m = rd.shape[0]
    cnt = ctypes.c_int(0)
    if with_pipes:
        pipes = np.zeros(3 * (m + 2), np.int32)
        npp = ctypes.c_int(0)
        acc = lib.or_sneakysnake(_p(rd), _p(rf), m, E, ctypes.byref(cnt), _p(pipes), m + 2,
                                 ctypes.byref(npp))
        lst = [tuple(int(x) for x in pipes[3 * i:3 * i + 3]) for i in range(npp.value)]
        return bool(acc), cnt.value, lst
    acc = lib.or_sneakysnake(_p(rd), _p(rf), m, E, ctypes.byref(cnt), None, 0, None)
    return bool(acc), cnt.value


def sneakysnake_weighted(read, ref, E):
    lib = _load()
    rd, rf = _u8(read), _u8(ref)
    cnt = ctypes.c_int(0)
    acc = lib.or_sneakysnake_weighted(_p(rd), _p(rf), rd.shape[0], E, ctypes.byref(cnt))
    return bool(acc), cnt.value


def sneakysnake_t(read, ref, E, t):
    """(accept, count) of SneakySnake on the maze cut into sub-mazes of t columns."""
    lib = _load()
    rd, rf = _u8(read), _u8(ref)
    cnt = ctypes.c_int(0)
    acc = lib.or_sneakysnake_t(_p(rd), _p(rf), rd.shape[0], E, t, ctypes.byref(cnt))
    return bool(acc), cnt.value


def sneakysnake_fpga(read, ref, E, t, y):
    """(accept, count) of the hardware form: sub-mazes of t columns, y replications each."""
    lib = _load()
    rd, rf = _u8(read), _u8(ref)
    cnt = ctypes.c_int(0)
    acc = lib.or_sneakysnake_fpga(_p(rd), _p(rf), rd.shape[0], E, t, y, ctypes.byref(cnt))
    return bool(acc), cnt.value


def sneakysnake_fpga_batch(reads, refs, lens, Es, t, y, threads=None):
    lib = _load()
    reads, refs = _u8(reads), _u8(refs)
    n, stride = reads.shape
    lens = np.ascontiguousarray(np.asarray(lens, np.uint16))
    Es = np.ascontiguousarray(np.broadcast_to(np.asarray(Es, np.uint8), (n,)))
    a = np.zeros(n, np.uint8)
    c = np.zeros(n, np.uint16)
    lib.or_sneakysnake_fpga_batch(_p(reads), _p(refs), stride, _p(lens), _p(Es), n, int(t), int(y), _p(a), _p(c),
                                  _threads(threads))
    return a, c


def magnet(read, ref, E, with_segments=False):
    """(accept, count[, segments]) of MAGNET; segments = [(diagonal, start, length)] in the order found."""
    lib = _load()
    rd, rf = _u8(read), _u8(ref)
    cnt = ctypes.c_int(0)
    segs = np.zeros(3 * (E + 1), np.int32)
    ns = ctypes.c_int(0)
    acc = lib.or_magnet(_p(rd), _p(rf), rd.shape[0], E, ctypes.byref(cnt), _p(segs), ctypes.byref(ns))
    if with_segments:
        return bool(acc), cnt.value, [tuple(int(x) for x in segs[3 * i:3 * i + 3]) for i in range(ns.value)]
    return bool(acc), cnt.value


def magnet_batch(reads, refs, lens, Es, threads=None):
    """(accept uint8[n], count uint16[n]) of MAGNET over a batch."""
    lib = _load()
    reads, refs = _u8(reads), _u8(refs)
    n, stride = reads.shape
    lens = np.ascontiguousarray(np.asarray(lens, np.uint16))
    Es = np.ascontiguousarray(np.broadcast_to(np.asarray(Es, np.uint8), (n,)))
    a = np.zeros(n, np.uint8)
    c = np.zeros(n, np.uint16)
    lib.or_magnet_batch(_p(reads), _p(refs), stride, _p(lens), _p(Es), n, _p(a), _p(c), _threads(threads))
    return a, c


def gatekeeper(read, ref, E):
    lib = _load()
    rd, rf = _u8(read), _u8(ref)
    cnt = ctypes.c_int(0)
    acc = lib.or_gatekeeper(_p(rd), _p(rf), rd.shape[0], E, ctypes.byref(cnt))
    return bool(acc), cnt.value


def shouji(read, ref, E, with_vector=False):
    lib = _load()
    rd, rf = _u8(read), _u8(ref)
    m = rd.shape[0]
    cnt = ctypes.c_int(0)
    S = np.zeros(max(m, 1), np.uint8)
    acc = lib.or_shouji(_p(rd), _p(rf), m, E, ctypes.byref(cnt), _p(S))
    if with_vector:
        return bool(acc), cnt.value, "".join(str(int(b)) for b in S[:m])
    return bool(acc), cnt.value


def amend(mask) -> np.ndarray:
    """GateKeeper/SHD amendment of one 0/1 mask."""
    lib = _load()
    x = _u8(mask)
    y = np.zeros_like(x)
    lib.or_amend(_p(x), _p(y), x.shape[0])
    return y


def banded_levenshtein(a, b, E):
    lib = _load()
    x, y = _u8(a), _u8(b)
    return lib.or_banded_levenshtein(_p(x), _p(y), x.shape[0], E)


def levenshtein(a, b):
    lib = _load()
    x, y = _u8(a), _u8(b)
    if x.shape[0] == 0 or y.shape[0] == 0:
        return int(max(x.shape[0], y.shape[0]))
    return lib.or_levenshtein(_p(x), x.shape[0], _p(y), y.shape[0])


def hamming(a, b):
    lib = _load()
    x, y = _u8(a), _u8(b)
    return lib.or_hamming(_p(x), _p(y), x.shape[0])


def features(read, ref, E) -> np.ndarray:
    lib = _load()
    rd, rf = _u8(read), _u8(ref)
    f = np.zeros(64, np.float64)
    lib.or_features(_p(rd), _p(rf), rd.shape[0], E, _p(f))
    return f


def _threads(threads):
    return threads or max(1, min(16, os.cpu_count() or 1))


def filter_batch(reads, refs, lens, Es, filters=SNEAKYSNAKE, threads=None):
    """Batch over pairs (rows of the [n, stride] uint8 arrays).  Returns a dict
    {filter bit: (accept uint8[n], count uint16[n])}."""
    lib = _load()
    reads, refs = _u8(reads), _u8(refs)
    n, stride = reads.shape
    lens = np.ascontiguousarray(np.asarray(lens, np.uint16))
    Es = np.ascontiguousarray(np.broadcast_to(np.asarray(Es, np.uint8), (n,)))
    out = {}
    bufs = []
    for f in (SNEAKYSNAKE, GATEKEEPER, SHOUJI):
        a = np.zeros(n, np.uint8)
        c = np.zeros(n, np.uint16)
        bufs += [_p(a) if filters & f else None, _p(c) if filters & f else None]
        if filters & f:
            out[f] = (a, c)
    lib.or_filter_batch(_p(reads), _p(refs), stride, _p(lens), _p(Es), n, filters, *bufs,
                        _threads(threads))
    return out


def sneakysnake_t_batch(reads, refs, lens, Es, t, threads=None):
    """(accept uint8[n], count uint16[n]) of SneakySnake-t over a batch."""
    lib = _load()
    reads, refs = _u8(reads), _u8(refs)
    n, stride = reads.shape
    lens = np.ascontiguousarray(np.asarray(lens, np.uint16))
    Es = np.ascontiguousarray(np.broadcast_to(np.asarray(Es, np.uint8), (n,)))
    a = np.zeros(n, np.uint8)
    c = np.zeros(n, np.uint16)
    lib.or_sneakysnake_t_batch(_p(reads), _p(refs), stride, _p(lens), _p(Es), n, int(t), _p(a), _p(c),
                               _threads(threads))
    return a, c


def banded_batch(reads, refs, lens, Es, threads=None) -> np.ndarray:
    lib = _load()
    reads, refs = _u8(reads), _u8(refs)
    n, stride = reads.shape
    lens = np.ascontiguousarray(np.asarray(lens, np.uint16))
    Es = np.ascontiguousarray(np.broadcast_to(np.asarray(Es, np.uint8), (n,)))
    d = np.zeros(n, np.uint16)
    lib.or_banded_batch(_p(reads), _p(refs), stride, _p(lens), _p(Es), n, _p(d), _threads(threads))
    return d


def features_batch(reads, refs, lens, Es, threads=None) -> np.ndarray:
    lib = _load()
    reads, refs = _u8(reads), _u8(refs)
    n, stride = reads.shape
    lens = np.ascontiguousarray(np.asarray(lens, np.uint16))
    Es = np.ascontiguousarray(np.broadcast_to(np.asarray(Es, np.uint8), (n,)))
    f = np.zeros((n, 64), np.float64)
    lib.or_features_batch(_p(reads), _p(refs), stride, _p(lens), _p(Es), n, _p(f), _threads(threads))
    return f
