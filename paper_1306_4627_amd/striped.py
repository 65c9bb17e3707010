"""Host baseline: the paper's row-striped OpenMP method (section II), built
from ``host/striped.c``.  Not part of the GPU path; it sets the paper's own
parallel algorithm, on this host's cores, beside the GPU numbers."""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstriped.so")


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1306_4627_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    u8p, u64 = ctypes.POINTER(ctypes.c_uint8), ctypes.c_uint64
    lib.striped_lcs.argtypes = [u8p, u64, u8p, u64, ctypes.c_int, ctypes.c_int, u8p,
                                ctypes.POINTER(u64), ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double)]
    lib.striped_lcs.restype = ctypes.c_int
    return lib


_lib = _load()


def _ptr(a: np.ndarray):
    if a.size == 0:
        return ctypes.POINTER(ctypes.c_uint8)()
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def striped_lcs(x, y, threads: int, chunk: int = 64, traceback: bool = True
                ) -> Tuple[int, Optional[bytes], float, float]:
    """(length, LCS bytes or None, fill seconds, total seconds)."""
    xa = np.ascontiguousarray(np.frombuffer(bytes(x), np.uint8) if isinstance(x, (bytes, bytearray))
                              else np.asarray(x, np.uint8))
    ya = np.ascontiguousarray(np.frombuffer(bytes(y), np.uint8) if isinstance(y, (bytes, bytearray))
                              else np.asarray(y, np.uint8))
    out = np.empty(max(1, min(xa.size, ya.size)), np.uint8) if traceback else None
    L = ctypes.c_uint64(0)
    tf = ctypes.c_double(0.0)
    tt = ctypes.c_double(0.0)
    st = _lib.striped_lcs(_ptr(xa), xa.size, _ptr(ya), ya.size, int(threads), int(chunk),
                          _ptr(out) if out is not None else ctypes.POINTER(ctypes.c_uint8)(),
                          ctypes.byref(L), ctypes.byref(tf), ctypes.byref(tt))
    if st != 0:
        raise RuntimeError(f"striped_lcs failed ({st})")
    s = out[: L.value].tobytes() if out is not None else None
    return int(L.value), s, float(tf.value), float(tt.value)
