"""Deliberately altered copies of the CPU oracle, for showing that a pin fails
when the rule it pins is changed.

`mutant(edits)` copies oracle/oracle.c, applies each (old, new) text edit
(each `old` must occur exactly once, so an edit cannot silently miss), builds
the copy with gcc into a temporary directory and, inside the `with` block,
points the oracle package's wrappers at that copy.  Only the tests use this;
the altered sources never leave the temporary directory."""
from __future__ import annotations

import contextlib
import os
import subprocess
import tempfile

import oracle

_SRC = os.path.join(os.path.dirname(os.path.abspath(oracle.__file__)), "oracle.c")
_cache: dict = {}


def _build(edits: tuple) -> str:
    if edits in _cache:
        return _cache[edits]
    src = open(_SRC).read()
    for old, new in edits:
        n = src.count(old)
        assert n == 1, f"mutation anchor found {n} times: {old!r}"
        src = src.replace(old, new)
    d = tempfile.mkdtemp(prefix="oracle_mutant_")
    c = os.path.join(d, "oracle.c")
    with open(c, "w") as f:
        f.write(src)
    so = os.path.join(d, "liboracle.so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", so, c])
    _cache[edits] = so
    return so


@contextlib.contextmanager
def mutant(*edits):
    """Run the oracle's wrappers on a copy of oracle.c with `edits` applied."""
    so = _build(tuple(edits))
    saved_lib, saved_path = oracle._lib, oracle._LIB
    oracle._lib, oracle._LIB = None, so
    try:
        yield
    finally:
        oracle._lib, oracle._LIB = saved_lib, saved_path
