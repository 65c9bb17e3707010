"""Python face of the CPU oracle (test infrastructure only).

The dynamic program itself lives in ``lcs_oracle.c`` (plain C, compiled with
gcc by ``build_oracle``).  This module adds the two exponential reference
methods the paper describes for tiny inputs, written in pure Python:

* ``brute_force_length`` -- section I (introduction) and I.A: enumerate every
  subsequence of X (2^m of them) and test each against Y in O(n).
* ``recursive_length`` -- section I.B: if the last symbols match, recurse on
  both prefixes and add one; otherwise take the larger of the two
  sub-problems.  No memoisation, exponential time.

Nothing here is used by, or uses, the GPU library.
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess
from typing import Iterable, Optional

import numpy as np

DIAG, UP, LEFT = 1, 2, 3

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lcs_oracle.c")
_LIB = os.path.join(_HERE, "liblcs_oracle.so")
_lib: Optional[ctypes.CDLL] = None


def build_oracle(force: bool = True) -> str:
    """Compile the C oracle with gcc into ``oracle/liblcs_oracle.so``.

    Built for the generic x86-64 target, so the shared object runs on any
    host the tree is copied to."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O3", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def use_native_build() -> str:
    """Rebuild the oracle with ``-O3 -march=native`` for the host this runs
    on and load that copy instead (for timing the oracle as a CPU baseline;
    the arithmetic is the same source).  Must be called before any other
    oracle call in the process."""
    global _lib, _LIB
    if _lib is not None:
        raise RuntimeError("use_native_build() must come before the first oracle call")
    native = os.path.join(_HERE, "liblcs_oracle_native.so")
    tmp = native + ".tmp"
    subprocess.check_call(
        ["gcc", "-O3", "-march=native", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC])
    os.replace(tmp, native)
    _LIB = native
    return native


def _load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_oracle(force=True)
        lib = ctypes.CDLL(_LIB)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i64 = ctypes.c_int64
        lib.oracle_lcs_table.argtypes = [u8p, i64, u8p, i64, u32p, u8p]
        lib.oracle_lcs_table.restype = ctypes.c_uint32
        lib.oracle_print_lcs.argtypes = [u8p, u8p, i64, i64, u8p]
        lib.oracle_print_lcs.restype = i64
        lib.oracle_lcs_length.argtypes = [u8p, i64, u8p, i64]
        lib.oracle_lcs_length.restype = i64
        lib.oracle_lcs_traceback.argtypes = [u8p, i64, u8p, i64, u8p]
        lib.oracle_lcs_traceback.restype = i64
        lib.oracle_lcs_traceback_ckpt.argtypes = [u8p, i64, u8p, i64, i64, u8p]
        lib.oracle_lcs_traceback_ckpt.restype = i64
        _lib = lib
    return _lib


def _buf(s) -> np.ndarray:
    if isinstance(s, (bytes, bytearray, memoryview)):
        a = np.frombuffer(bytes(s), dtype=np.uint8)
    else:
        a = np.asarray(s, dtype=np.uint8)
    a = np.ascontiguousarray(a)
    if a.size == 0:
        a = np.zeros(1, dtype=np.uint8)[:0]
    return a


def _ptr(a: np.ndarray):
    if a.size == 0:
        return ctypes.cast(ctypes.create_string_buffer(1), ctypes.POINTER(ctypes.c_uint8))
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def lcs_tables(x, y):
    """Full c and b tables of section I.C as numpy arrays of shape (m+1, n+1)."""
    lib = _load()
    xa, ya = _buf(x), _buf(y)
    m, n = xa.size, ya.size
    c = np.zeros((m + 1, n + 1), dtype=np.uint32)
    b = np.zeros((m + 1, n + 1), dtype=np.uint8)
    lib.oracle_lcs_table(_ptr(xa), m, _ptr(ya), n,
                         c.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                         b.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return c, b


def lcs_length(x, y) -> int:
    """c[m][n] of section I.C (two-row storage, same recurrence)."""
    lib = _load()
    xa, ya = _buf(x), _buf(y)
    r = lib.oracle_lcs_length(_ptr(xa), xa.size, _ptr(ya), ya.size)
    if r < 0:
        raise MemoryError("oracle_lcs_length: allocation failed")
    return int(r)


def lcs_traceback(x, y) -> bytes:
    """Canonical LCS: full tables of section I.C walked per section I.D."""
    lib = _load()
    xa, ya = _buf(x), _buf(y)
    out = np.zeros(max(1, min(xa.size, ya.size)), dtype=np.uint8)
    r = lib.oracle_lcs_traceback(_ptr(xa), xa.size, _ptr(ya), ya.size, _ptr(out))
    if r < 0:
        raise MemoryError("oracle_lcs_traceback: allocation failed")
    return out[:r].tobytes()


def lcs_traceback_ckpt(x, y, rows_per_block: int = 512) -> bytes:
    """Canonical LCS with checkpointed rows (for tables too large to hold)."""
    lib = _load()
    xa, ya = _buf(x), _buf(y)
    out = np.zeros(max(1, min(xa.size, ya.size)), dtype=np.uint8)
    r = lib.oracle_lcs_traceback_ckpt(_ptr(xa), xa.size, _ptr(ya), ya.size,
                                      int(rows_per_block), _ptr(out))
    if r == -2:
        raise ValueError("rows_per_block must be >= 1")
    if r < 0:
        raise MemoryError("oracle_lcs_traceback_ckpt: allocation failed")
    return out[:r].tobytes()


# ---------------------------------------------------------------------------
# Derived outputs of section II: how much of the parent the child keeps.
# ---------------------------------------------------------------------------

def similarity_percent(x, y) -> float:
    """Section II asks whether the child (Y) carries the parent's (X)
    characteristics and by what percentage.  Reading: the share of the parent
    kept by the LCS, 100 * L / |X|, evaluated in double as (100 * L) / m
    (the product is exact).  An empty parent is kept whole: 100."""
    m = len(x)
    if m == 0:
        return 100.0
    return (100.0 * lcs_length(x, y)) / float(m)


def threshold_pass(x, y, min_percent: float) -> bool:
    """Section II's yes/no question for a threshold: does the child keep at
    least ``min_percent`` of the parent, i.e. similarity_percent >= it."""
    return similarity_percent(x, y) >= float(min_percent)


# ---------------------------------------------------------------------------
# Exponential reference methods for tiny inputs (pure Python).
# ---------------------------------------------------------------------------

def is_subsequence(z: bytes, s: bytes) -> bool:
    """True when z can be obtained from s by deleting symbols (O(|s|))."""
    it = iter(s)
    return all(any(ch == c for c in it) for ch in z)


def _subsequences_by_size(x: bytes) -> Iterable[bytes]:
    m = len(x)
    for size in range(m, -1, -1):
        for idx in itertools.combinations(range(m), size):
            yield bytes(x[i] for i in idx)


def brute_force_length(x: bytes, y: bytes) -> int:
    """Longest subsequence of X that is also a subsequence of Y, by trying
    every subsequence of X from the longest down (section I, brute force)."""
    x, y = bytes(x), bytes(y)
    if len(x) > 16:
        raise ValueError("brute force is limited to |X| <= 16")
    for z in _subsequences_by_size(x):
        if is_subsequence(z, y):
            return len(z)
    return 0


def brute_force_all_lcs(x: bytes, y: bytes) -> set:
    """Every distinct longest common subsequence, by enumeration."""
    x, y = bytes(x), bytes(y)
    if len(x) > 16:
        raise ValueError("brute force is limited to |X| <= 16")
    best, found = -1, set()
    for z in _subsequences_by_size(x):
        if best >= 0 and len(z) < best:
            break
        if is_subsequence(z, y):
            best = len(z)
            found.add(z)
    return found


def recursive_length(x: bytes, y: bytes) -> int:
    """Section I.B recursion on prefixes, without memoisation."""
    x, y = bytes(x), bytes(y)

    def rec(i: int, j: int) -> int:
        if i == 0 or j == 0:
            return 0
        if x[i - 1] == y[j - 1]:
            return rec(i - 1, j - 1) + 1
        return max(rec(i - 1, j), rec(i, j - 1))

    return rec(len(x), len(y))
