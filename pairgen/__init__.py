"""Seeded synthetic workloads of (read, reference segment) pairs.

Shared by the CPU oracle's tests and by the GPU path's tests and benchmark;
it holds none of the filtering method's arithmetic, only random DNA.  Every
pair is a pure function of (seed, pair id), so single pairs of a large batch
can be regenerated for sampled checks.  Bases are uint8 codes 0..3 (A, C, G, T).

The named workloads mirror the shapes of the thesis's evaluation sets (read
lengths of 100, 150 and 250 bp, thresholds from 0 up to 10% of the length,
mostly-incorrect candidate pairs; Ch. 9, experimental setup).  The real read
sets and genome are not available, so i.i.d. uniform bases and uniform random
edits stand in for them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pairgen.c")
_LIB = os.path.join(_HERE, "libpairgen.so")

SEED_BASE = 1910_03936


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64),
        ("n_len", ctypes.c_uint32),
        ("lens", ctypes.c_uint16 * 8),
        ("kmax", ctypes.c_uint32),
        ("unrelated", ctypes.c_double),
        ("fixed_E", ctypes.c_int32),
        ("e_num", ctypes.c_uint32),
        ("e_den", ctypes.c_uint32),
    ]


@dataclass(frozen=True)
class Workload:
    """A synthetic workload: lengths, edit count range, unrelated fraction, E rule."""
    name: str
    n_pairs: int
    lens: tuple
    kmax: int
    unrelated: float
    fixed_E: int = -1          # >= 0: uniform E
    e_num: int = 0             # fixed_E < 0: E = floor(m * e_num / e_den)
    e_den: int = 1
    seed: int = SEED_BASE

    @property
    def max_len(self) -> int:
        return max(self.lens)

    def with_E(self, E: int) -> "Workload":
        return Workload(self.name, self.n_pairs, self.lens, self.kmax, self.unrelated, E,
                        self.e_num, self.e_den, self.seed)

    def with_n(self, n: int) -> "Workload":
        return Workload(self.name, n, self.lens, self.kmax, self.unrelated, self.fixed_E,
                        self.e_num, self.e_den, self.seed)

    def with_seed(self, seed: int) -> "Workload":
        return Workload(self.name, self.n_pairs, self.lens, self.kmax, self.unrelated, self.fixed_E,
                        self.e_num, self.e_den, seed)

    def _cfg(self) -> _Cfg:
        c = _Cfg()
        c.seed = self.seed
        c.n_len = len(self.lens)
        for i, m in enumerate(self.lens):
            c.lens[i] = m
        c.kmax = self.kmax
        c.unrelated = self.unrelated
        c.fixed_E = self.fixed_E
        c.e_num = self.e_num
        c.e_den = self.e_den
        return c


# The five workloads.  Seeds differ per workload so that their pairs differ.
SMALL_100BP = Workload("100bp, E=5, 100k pairs, 50% unrelated, k<=15", 100_000, (100,), 15, 0.5,
                       fixed_E=5, seed=SEED_BASE + 0)
FIXED_250BP = Workload("250bp, 10M pairs, 70% unrelated, k<=40", 10_000_000, (250,), 40, 0.7,
                       fixed_E=10, seed=SEED_BASE + 1)
UNEVEN_MIX = Workload("lengths {64,100,150,250,300}, E=floor(0.05 m), 50M pairs, 70% unrelated, k<=40",
                      50_000_000, (64, 100, 150, 250, 300), 40, 0.7, e_num=5, e_den=100,
                      seed=SEED_BASE + 2)
TRAIN_MIX = Workload("MLP training pairs drawn like the uneven mix, 2M pairs", 2_000_000,
                     (64, 100, 150, 250, 300), 40, 0.7, e_num=5, e_den=100, seed=SEED_BASE + 3)
STREAM_MIX = Workload("lengths {100,150,250} 1:1:1, E=m/10, 200M pairs, 80% unrelated, k<=40",
                      200_000_000, (100, 150, 250), 40, 0.8, e_num=10, e_den=100, seed=SEED_BASE + 4)

WORKLOADS = {"small": SMALL_100BP, "fixed250": FIXED_250BP, "uneven": UNEVEN_MIX,
             "train": TRAIN_MIX, "stream": STREAM_MIX}


def build(force: bool = False) -> str:
    """Compile libpairgen.so with gcc (host code only)."""
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
        P = ctypes.c_void_p
        lib.pg_generate.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_uint64, ctypes.c_uint64, P, P,
                                    ctypes.c_uint32, P, P, P, P, ctypes.c_int]
        lib.pg_generate.restype = ctypes.c_int
        lib.pg_generate_ids.argtypes = [ctypes.POINTER(_Cfg), P, ctypes.c_uint64, P, P,
                                        ctypes.c_uint32, P, P, P, P, ctypes.c_int]
        lib.pg_generate_ids.restype = ctypes.c_int
        lib.pg_lengths.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_uint64, ctypes.c_uint64, P, P, ctypes.c_int]
        lib.pg_lengths.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Pairs:
    """A batch of generated pairs: reads/refs are [n, stride] uint8 codes, row i
    valid up to len[i]; E, related and k (edits applied) per pair."""
    reads: np.ndarray
    refs: np.ndarray
    len: np.ndarray
    E: np.ndarray
    related: np.ndarray
    k: np.ndarray
    ids: np.ndarray = field(default=None)

    @property
    def n(self) -> int:
        return int(self.len.shape[0])

    @property
    def stride(self) -> int:
        return int(self.reads.shape[1])


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def generate(w: Workload, first: int = 0, n: int | None = None, stride: int | None = None,
             threads: int | None = None) -> Pairs:
    """Pairs [first, first + n) of workload w."""
    lib = _load()
    n = w.n_pairs - first if n is None else n
    stride = w.max_len if stride is None else stride
    reads = np.zeros((n, stride), np.uint8)
    refs = np.zeros((n, stride), np.uint8)
    ln = np.zeros(n, np.uint16)
    E = np.zeros(n, np.uint8)
    rel = np.zeros(n, np.uint8)
    k = np.zeros(n, np.uint16)
    cfg = w._cfg()
    rc = lib.pg_generate(ctypes.byref(cfg), first, n, _ptr(reads), _ptr(refs), stride,
                         _ptr(ln), _ptr(E), _ptr(rel), _ptr(k), threads or default_threads())
    if rc != 0:
        raise ValueError(f"pairgen rejected workload {w}")
    return Pairs(reads, refs, ln, E, rel, k, np.arange(first, first + n, dtype=np.uint64))


def generate_ids(w: Workload, ids, stride: int | None = None, threads: int | None = None) -> Pairs:
    """The pairs of workload w with the given ids (any order, repeats allowed)."""
    lib = _load()
    ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint64))
    n = ids.shape[0]
    stride = w.max_len if stride is None else stride
    reads = np.zeros((n, stride), np.uint8)
    refs = np.zeros((n, stride), np.uint8)
    ln = np.zeros(n, np.uint16)
    E = np.zeros(n, np.uint8)
    rel = np.zeros(n, np.uint8)
    k = np.zeros(n, np.uint16)
    cfg = w._cfg()
    rc = lib.pg_generate_ids(ctypes.byref(cfg), _ptr(ids), n, _ptr(reads), _ptr(refs), stride,
                             _ptr(ln), _ptr(E), _ptr(rel), _ptr(k), threads or default_threads())
    if rc != 0:
        raise ValueError(f"pairgen rejected workload {w}")
    return Pairs(reads, refs, ln, E, rel, k, ids)


def lengths(w: Workload, first: int = 0, n: int | None = None, threads: int | None = None):
    """(len uint16[n], E uint8[n]) of pairs [first, first + n) without their bases."""
    lib = _load()
    n = w.n_pairs - first if n is None else n
    ln = np.zeros(n, np.uint16)
    E = np.zeros(n, np.uint8)
    cfg = w._cfg()
    if lib.pg_lengths(ctypes.byref(cfg), first, n, _ptr(ln), _ptr(E), threads or default_threads()) != 0:
        raise ValueError(f"pairgen rejected workload {w}")
    return ln, E


def sample_ids(n_pairs: int, n_sample: int, seed: int = 7) -> np.ndarray:
    """A deterministic sorted sample of pair ids that always includes the first
    and last pair (the ragged tail)."""
    rng = np.random.default_rng(seed)
    n_sample = min(n_sample, n_pairs)
    ids = rng.choice(n_pairs, size=n_sample, replace=False).astype(np.uint64)
    ids = np.unique(np.concatenate([ids, np.array([0, n_pairs - 1], np.uint64)]))
    return ids


BASES = "ACGT"


def encode(s: str) -> np.ndarray:
    """ASCII A/C/G/T string -> uint8 codes (for hand-written examples)."""
    return np.array([BASES.index(ch) for ch in s], np.uint8)


def decode(codes) -> str:
    return "".join(BASES[int(c)] for c in codes)


def init_mlp_params(seed: int = SEED_BASE + 17) -> np.ndarray:
    """Seeded initial weights of the 64 -> 128 -> 128 -> 1 cost model (flat
    fp32, layout W1[128][64], b1[128], W2[128][128], b2[128], W3[128], b3):
    He-uniform weight matrices U(-sqrt(6 / fan_in), +sqrt(6 / fan_in)), zero
    biases.  Random numbers only, so both sides take them as input."""
    rng = np.random.default_rng(seed)
    parts = []
    for rows, fan_in in ((128, 64), (128, 128), (1, 128)):
        a = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-a, a, rows * fan_in))
        parts.append(np.zeros(rows))
    return np.concatenate(parts).astype(np.float32)
