"""Oracle: Levenshtein distance (§1: minimal number of insertions, deletions and
substitutions turning one string into another).

TEST INFRASTRUCTURE ONLY (see the package docstring).

`levenshtein` is the textbook dynamic programme in plain Python; `lev_many`
runs the same programme in plain C (oracle/levenshtein.c) for bulk labels;
`levenshtein_brute` finds the distance by breadth-first search over edit
scripts, for tiny strings only.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_liblev.so")
_lib = None


def levenshtein(a, b) -> int:
    a = [int(x) for x in a]
    b = [int(x) for x in b]
    prev = list(range(len(b) + 1))
    for i in range(1, len(a) + 1):
        cur = [i] + [0] * len(b)
        for j in range(1, len(b) + 1):
            cur[j] = min(prev[j] + 1, cur[j - 1] + 1, prev[j - 1] + (a[i - 1] != b[j - 1]))
        prev = cur
    return prev[len(b)]


def levenshtein_brute(a, b, alphabet=(0, 1, 2, 3)) -> int:
    """Smallest number of single-letter edits reaching b from a, by BFS."""
    a, b = tuple(int(x) for x in a), tuple(int(x) for x in b)
    if a == b:
        return 0
    frontier, seen, d = {a}, {a}, 0
    limit = len(b) + len(a) + 1
    while frontier:
        d += 1
        nxt = set()
        for s in frontier:
            cand = []
            for i in range(len(s)):
                cand.append(s[:i] + s[i + 1:])
                for c in alphabet:
                    if c != s[i]:
                        cand.append(s[:i] + (c,) + s[i + 1:])
            for i in range(len(s) + 1):
                if len(s) < limit:
                    for c in alphabet:
                        cand.append(s[:i] + (c,) + s[i:])
            for t in cand:
                if t == b:
                    return d
                if t not in seen:
                    seen.add(t)
                    nxt.add(t)
        frontier = nxt
    raise RuntimeError("unreachable")


def build(cc: str = "gcc") -> str:
    import subprocess
    src = os.path.join(_HERE, "levenshtein.c")
    subprocess.check_call([cc, "-O2", "-shared", "-fPIC", "-o", _LIB_PATH, src])
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        p = ctypes.c_void_p
        lib.lev_many.argtypes = [p, p, p, p, ctypes.c_int64, p]
        lib.lev_many.restype = ctypes.c_int
        _lib = lib
    return _lib


def lev_many(a: np.ndarray, a_off: np.ndarray, b: np.ndarray, b_off: np.ndarray) -> np.ndarray:
    """Distances of all pairs (concatenated uint8 strings with int64 offsets)."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    a_off = np.ascontiguousarray(a_off, dtype=np.int64)
    b_off = np.ascontiguousarray(b_off, dtype=np.int64)
    n = a_off.shape[0] - 1
    out = np.zeros(n, dtype=np.int64)
    rc = lib.lev_many(a.ctypes.data, a_off.ctypes.data, b.ctypes.data, b_off.ctypes.data, n, out.ctypes.data)
    if rc != 0:
        raise MemoryError("lev_many")
    return out
