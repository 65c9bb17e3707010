"""Thin ctypes binding of ``liblcs_hip.so`` (C ABI in ``include/lcs.h``).

Argument marshalling only: every step of the LCS computation runs in the
library's gfx950 kernels.  The library must have been built
(``python -m paper_1306_4627_amd.build`` or ``__graft_entry__.build()``);
importing this module without it raises ``ImportError`` -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblcs_hip.so")

LCS_PENDING = 1
LCS_OK = 0
LCS_ERR_ARG = -1
LCS_ERR_SYMBOL = -2
LCS_ERR_NOMEM = -3
LCS_ERR_DEVICE = -4
LCS_ERR_BUFFER = -5
LCS_ERR_TOO_LONG = -6
LCS_ERR_UNSUPPORTED = -7

LCS_WANT_TRACEBACK = 1
LCS_USE_GRAPH = 2
LCS_THRESHOLD = 4
LCS_FILL_TRACE = 8
LCS_LENGTH_UNKNOWN = (1 << 64) - 1

# lcs_fill_item
FILL_ITEM = np.dtype([("start_ns", "<u8"), ("first_step_ns", "<u8"), ("end_ns", "<u8"),
                      ("wait_ns", "<u8"), ("steps", "<u4"), ("feeder", "<i4"), ("feeds", "<u4"),
                      ("ran", "<u4"), ("hw_id", "<u4"), ("xcc_id", "<u4")])

DNA = b"ACGT"
PROTEIN = b"ACDEFGHIKLMNPQRSTVWY"


class LcsError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        detail = ""
        if status in (LCS_ERR_DEVICE, LCS_ERR_NOMEM):
            detail = " [" + _lib.lcs_last_error().decode(errors="replace") + "]"
        msg = f"{what}: {status_str(status)} ({status})" if what else status_str(status)
        super().__init__(msg + detail)


class lcs_alphabet(ctypes.Structure):
    _fields_ = [("size", ctypes.c_uint16), ("symbols", ctypes.POINTER(ctypes.c_uint8))]


class lcs_pair(ctypes.Structure):
    _fields_ = [("x", ctypes.POINTER(ctypes.c_uint8)), ("m", ctypes.c_uint64),
                ("y", ctypes.POINTER(ctypes.c_uint8)), ("n", ctypes.c_uint64)]


class lcs_tuning(ctypes.Structure):
    _fields_ = [("words_per_lane", ctypes.c_int32), ("ckpt_interval", ctypes.c_int32),
                ("persistent_waves", ctypes.c_int32), ("plain", ctypes.c_int32),
                ("strip_rows", ctypes.c_int32), ("tb_tiles", ctypes.c_int32),
                ("tb_bands", ctypes.c_int32), ("link_items", ctypes.c_int32),
                ("tb_round_kib", ctypes.c_int32), ("halves", ctypes.c_int32)]


class lcs_server_config(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_size_t), ("streams", ctypes.c_int32),
                ("max_batch_pairs", ctypes.c_int32)]


class lcs_server_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("submitted", "completed", "failed", "cancelled",
                                                "queued", "batches", "max_inflight", "cells",
                                                "arena_bytes", "arena_peak_bytes", "plan_ns",
                                                "collect_ns", "device_ns", "tuned_batches")]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class lcs_batch_stats(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_uint64), ("cells", ctypes.c_uint64),
                ("groups", ctypes.c_uint64), ("lanes", ctypes.c_uint64),
                ("lane_steps", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64),
                ("words_per_lane", ctypes.c_int32), ("ckpt_interval", ctypes.c_int32),
                ("classes", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("tb_rounds", ctypes.c_int32), ("split_pairs", ctypes.c_int32),
                ("history_bytes", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1306_4627_amd/build.py "
                          "(no CPU fallback exists)")
    # One HIP runtime per process.  PyTorch ships its own libamdhip64 and
    # links it under another name than this library's; loaded first, it
    # satisfies this library's dependency too, so device memory and streams
    # are shared and the device is never opened by two runtimes.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    u8p, u64p, vp = P(ctypes.c_uint8), P(ctypes.c_uint64), ctypes.c_void_p
    u64, i32 = ctypes.c_uint64, ctypes.c_int
    lib.lcs_status_str.argtypes = [i32]
    lib.lcs_status_str.restype = ctypes.c_char_p
    lib.lcs_version.argtypes = []
    lib.lcs_version.restype = ctypes.c_char_p
    lib.lcs_last_error.argtypes = []
    lib.lcs_last_error.restype = ctypes.c_char_p
    lib.lcs_create.argtypes = [P(vp), i32, ctypes.c_size_t]
    lib.lcs_create.restype = i32
    lib.lcs_destroy.argtypes = [vp]
    lib.lcs_destroy.restype = None
    lib.lcs_device_info.argtypes = [vp, P(ctypes.c_int32), P(ctypes.c_int32)]
    lib.lcs_device_info.restype = i32
    lib.lcs_set_stream.argtypes = [vp, vp]
    lib.lcs_set_stream.restype = i32
    lib.lcs_synchronize.argtypes = [vp]
    lib.lcs_synchronize.restype = i32
    lib.lcs_length.argtypes = [vp, u8p, u64, u8p, u64, P(lcs_alphabet), u64p]
    lib.lcs_length.restype = i32
    lib.lcs_traceback.argtypes = [vp, u8p, u64, u8p, u64, P(lcs_alphabet), u8p, u64, u64p]
    lib.lcs_traceback.restype = i32
    lib.lcs_length_batch.argtypes = [vp, P(lcs_pair), u64, P(lcs_alphabet), u64p]
    lib.lcs_length_batch.restype = i32
    lib.lcs_traceback_batch.argtypes = [vp, P(lcs_pair), u64, P(lcs_alphabet), u8p, u64,
                                        u64p, u64p]
    lib.lcs_traceback_batch.restype = i32
    lib.lcs_traceback_batch_noalloc.argtypes = [vp, P(lcs_pair), u64, P(lcs_alphabet), u8p, u64,
                                                u64p, u64p]
    lib.lcs_traceback_batch_noalloc.restype = i32
    lib.lcs_noalloc_scratch_bytes.argtypes = []
    lib.lcs_noalloc_scratch_bytes.restype = u64
    lib.lcs_batch_create.argtypes = [vp, P(lcs_pair), u64, P(lcs_alphabet), ctypes.c_uint32,
                                     P(lcs_tuning), P(vp)]
    lib.lcs_batch_create.restype = i32
    lib.lcs_batch_run.argtypes = [vp]
    lib.lcs_batch_run.restype = i32
    lib.lcs_batch_lengths.argtypes = [vp, u64p]
    lib.lcs_batch_lengths.restype = i32
    lib.lcs_batch_tracebacks.argtypes = [vp, u8p, u64, u64p, u64p]
    lib.lcs_batch_tracebacks.restype = i32
    lib.lcs_batch_info.argtypes = [vp, P(lcs_batch_stats)]
    lib.lcs_batch_info.restype = i32
    lib.lcs_batch_time.argtypes = [vp, i32, P(ctypes.c_float), P(ctypes.c_float)]
    lib.lcs_batch_time.restype = i32
    lib.lcs_batch_destroy.argtypes = [vp]
    lib.lcs_batch_destroy.restype = None
    lib.lcs_autotune.argtypes = [vp, P(lcs_pair), u64, P(lcs_alphabet), ctypes.c_uint32,
                                 P(lcs_tuning), P(ctypes.c_float)]
    lib.lcs_autotune.restype = i32
    lib.lcs_similarity_batch.argtypes = [vp, P(lcs_pair), u64, P(lcs_alphabet),
                                         P(ctypes.c_double)]
    lib.lcs_similarity_batch.restype = i32
    lib.lcs_threshold_batch.argtypes = [vp, P(lcs_pair), u64, P(lcs_alphabet), ctypes.c_double,
                                        u8p, u64p]
    lib.lcs_threshold_batch.restype = i32
    lib.lcs_batch_set_threshold.argtypes = [vp, ctypes.c_double]
    lib.lcs_batch_set_threshold.restype = i32
    lib.lcs_batch_decisions.argtypes = [vp, u8p, u64p]
    lib.lcs_batch_decisions.restype = i32
    lib.lcs_batch_clock.argtypes = [vp, P(ctypes.c_double)]
    lib.lcs_batch_clock.restype = i32
    lib.lcs_batch_fill_trace.argtypes = [vp, vp, u64, u64p]
    lib.lcs_batch_fill_trace.restype = i32
    lib.lcs_server_create.argtypes = [vp, P(lcs_server_config), P(vp)]
    lib.lcs_server_create.restype = i32
    lib.lcs_server_destroy.argtypes = [vp]
    lib.lcs_server_destroy.restype = None
    lib.lcs_submit.argtypes = [vp, u8p, u64, u8p, u64, P(lcs_alphabet), i32, u64p]
    lib.lcs_submit.restype = i32
    lib.lcs_poll.argtypes = [vp, u64]
    lib.lcs_poll.restype = i32
    lib.lcs_wait.argtypes = [vp, u64, ctypes.c_int64]
    lib.lcs_wait.restype = i32
    lib.lcs_result.argtypes = [vp, u64, u64p, u8p, u64, u64p]
    lib.lcs_result.restype = i32
    lib.lcs_cancel.argtypes = [vp, u64]
    lib.lcs_cancel.restype = i32
    lib.lcs_server_stats_get.argtypes = [vp, P(lcs_server_stats)]
    lib.lcs_server_stats_get.restype = i32
    lib.lcs_plan_describe.argtypes = [u64p, u64p, u64, ctypes.c_uint16, ctypes.c_uint32,
                                      P(lcs_tuning), P(lcs_batch_stats)]
    lib.lcs_plan_describe.restype = i32
    lib.lcs_plan_selfcheck.argtypes = [u64p, u64p, u64, ctypes.c_uint16, ctypes.c_uint32,
                                       P(lcs_tuning)]
    lib.lcs_plan_selfcheck.restype = i32
    return lib


_lib = _load()


def lib() -> ctypes.CDLL:
    return _lib


def status_str(status: int) -> str:
    return _lib.lcs_status_str(int(status)).decode()


def version() -> str:
    return _lib.lcs_version().decode()


def _check(status: int, what: str) -> None:
    if status != LCS_OK:
        raise LcsError(status, what)


def _as_u8(s) -> np.ndarray:
    if isinstance(s, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(s), dtype=np.uint8)
    return np.ascontiguousarray(np.asarray(s, dtype=np.uint8))


def _u8p(a: np.ndarray):
    if a.size == 0:
        return ctypes.POINTER(ctypes.c_uint8)()
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


class Alphabet:
    """An alphabet (``bytes`` of distinct symbols, or None for all 256 bytes)."""

    def __init__(self, symbols: Optional[bytes]):
        if symbols is None:
            self._buf = None
            self.c = lcs_alphabet(256, ctypes.POINTER(ctypes.c_uint8)())
        else:
            self._buf = np.frombuffer(bytes(symbols), dtype=np.uint8).copy()
            self.c = lcs_alphabet(len(symbols), _u8p(self._buf))

    @property
    def size(self) -> int:
        return int(self.c.size)


def _alpha(a) -> Alphabet:
    if isinstance(a, Alphabet):
        return a
    if a is None or a == "byte":
        return Alphabet(None)
    if isinstance(a, str):
        return Alphabet({"dna": DNA, "protein": PROTEIN}[a])
    return Alphabet(bytes(a))


def _tuning(words_per_lane=0, ckpt_interval=0, persistent_waves=0, plain=False, strip_rows=0,
            tb_tiles=0, tb_bands=0, link_items=0, tb_round_kib=0, halves=0):
    return lcs_tuning(int(words_per_lane), int(ckpt_interval), int(persistent_waves), int(bool(plain)),
                      int(strip_rows), int(tb_tiles), int(tb_bands), int(link_items),
                      int(tb_round_kib), int(halves))


class _Pairs:
    """Keeps the numpy buffers alive while the C array points into them."""

    def __init__(self, pairs: Sequence[Tuple[object, object]]):
        self.bufs = []
        self.count = len(pairs)
        # the lcs_pair array as one record array: {x, m, y, n}, 8 bytes each
        words = []
        for x, y in pairs:
            xa, ya = _as_u8(x), _as_u8(y)
            self.bufs += [xa, ya]
            words += [xa.__array_interface__["data"][0] if xa.size else 0, xa.size,
                      ya.__array_interface__["data"][0] if ya.size else 0, ya.size]
        self.rec = np.array(words if words else [0, 0, 0, 0], dtype=np.uint64)
        m = self.rec[1::4]
        n = self.rec[3::4]
        # sum of min(m, n): the output capacity of the strings
        self.cap = int(np.minimum(m, n).sum()) if self.count else 0

    def ptr(self):
        if not self.count:
            return ctypes.POINTER(lcs_pair)()
        return ctypes.cast(self.rec.ctypes.data, ctypes.POINTER(lcs_pair))


class Context:
    """One device, one stream, a device-memory budget (``lcs_create``)."""

    def __init__(self, device: int = 0, mem_budget_bytes: int = 0):
        h = ctypes.c_void_p()
        _check(_lib.lcs_create(ctypes.byref(h), int(device), int(mem_budget_bytes)), "lcs_create")
        self.h = h

    def close(self) -> None:
        if self.h:
            _lib.lcs_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def device_info(self) -> dict:
        """Compute units and peak shader clock (kHz) of the context's device."""
        cu, clk = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(_lib.lcs_device_info(self.h, ctypes.byref(cu), ctypes.byref(clk)), "lcs_device_info")
        return {"compute_units": int(cu.value), "peak_clock_khz": int(clk.value)}

    def set_stream(self, stream) -> None:
        """Use a HIP stream: an int handle, a ``torch.cuda.Stream`` or None."""
        handle = None
        if stream is not None:
            handle = getattr(stream, "cuda_stream", stream)
        _check(_lib.lcs_set_stream(self.h, ctypes.c_void_p(handle) if handle else None),
               "lcs_set_stream")

    def synchronize(self) -> None:
        _check(_lib.lcs_synchronize(self.h), "lcs_synchronize")


def lcs_length(ctx: Context, x, y, alphabet="dna") -> int:
    xa, ya = _as_u8(x), _as_u8(y)
    al = _alpha(alphabet)
    out = ctypes.c_uint64()
    _check(_lib.lcs_length(ctx.h, _u8p(xa), xa.size, _u8p(ya), ya.size, ctypes.byref(al.c),
                           ctypes.byref(out)), "lcs_length")
    return int(out.value)


def lcs_traceback(ctx: Context, x, y, alphabet="dna") -> bytes:
    xa, ya = _as_u8(x), _as_u8(y)
    al = _alpha(alphabet)
    cap = min(xa.size, ya.size)
    buf = np.zeros(max(1, cap), dtype=np.uint8)
    out = ctypes.c_uint64()
    _check(_lib.lcs_traceback(ctx.h, _u8p(xa), xa.size, _u8p(ya), ya.size, ctypes.byref(al.c),
                              _u8p(buf), cap, ctypes.byref(out)), "lcs_traceback")
    return buf[:out.value].tobytes()


def lcs_length_batch(ctx: Context, pairs, alphabet="dna") -> np.ndarray:
    pp = _Pairs(pairs)
    al = _alpha(alphabet)
    out = np.zeros(max(1, pp.count), dtype=np.uint64)
    _check(_lib.lcs_length_batch(ctx.h, pp.ptr(), pp.count, ctypes.byref(al.c),
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))),
           "lcs_length_batch")
    return out[:pp.count]


def lcs_traceback_batch(ctx: Context, pairs, alphabet="dna") -> List[bytes]:
    pp = _Pairs(pairs)
    al = _alpha(alphabet)
    cap = pp.cap
    arena = np.empty(max(1, cap), dtype=np.uint8)   # written where read back
    offs = np.zeros(max(1, pp.count), dtype=np.uint64)
    lens = np.zeros(max(1, pp.count), dtype=np.uint64)
    P64 = ctypes.POINTER(ctypes.c_uint64)
    _check(_lib.lcs_traceback_batch(ctx.h, pp.ptr(), pp.count, ctypes.byref(al.c), _u8p(arena),
                                    cap, offs.ctypes.data_as(P64), lens.ctypes.data_as(P64)),
           "lcs_traceback_batch")
    return [arena[int(o):int(o) + int(l)].tobytes() for o, l in zip(offs[:pp.count], lens[:pp.count])]


def lcs_traceback_batch_noalloc(ctx: Context, pairs, alphabet="dna") -> List[bytes]:
    """lcs_traceback_batch with every device buffer carved from the library's
    fixed device scratch array (no device allocation)."""
    pp = _Pairs(pairs)
    al = _alpha(alphabet)
    cap = pp.cap
    arena = np.empty(max(1, cap), dtype=np.uint8)   # written where read back
    offs = np.zeros(max(1, pp.count), dtype=np.uint64)
    lens = np.zeros(max(1, pp.count), dtype=np.uint64)
    P64 = ctypes.POINTER(ctypes.c_uint64)
    _check(_lib.lcs_traceback_batch_noalloc(ctx.h, pp.ptr(), pp.count, ctypes.byref(al.c),
                                            _u8p(arena), cap, offs.ctypes.data_as(P64),
                                            lens.ctypes.data_as(P64)),
           "lcs_traceback_batch_noalloc")
    return [arena[int(o):int(o) + int(l)].tobytes() for o, l in zip(offs[:pp.count], lens[:pp.count])]


def noalloc_scratch_bytes() -> int:
    return int(_lib.lcs_noalloc_scratch_bytes())


def lcs_similarity_batch(ctx: Context, pairs, alphabet="dna") -> np.ndarray:
    """Similarity percentages (100 * L) / |X| of each pair (100 for empty X)."""
    pp = _Pairs(pairs)
    al = _alpha(alphabet)
    out = np.zeros(max(1, pp.count), dtype=np.float64)
    _check(_lib.lcs_similarity_batch(ctx.h, pp.ptr(), pp.count, ctypes.byref(al.c),
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "lcs_similarity_batch")
    return out[:pp.count]


def lcs_threshold_batch(ctx: Context, pairs, min_percent: float,
                        alphabet="dna") -> Tuple[np.ndarray, np.ndarray]:
    """(pass, lengths): pass[k] is True when the similarity of pair k is at
    least min_percent; lengths[k] is its LCS length, or LCS_LENGTH_UNKNOWN
    when the answer came before the last column."""
    pp = _Pairs(pairs)
    al = _alpha(alphabet)
    ok = np.zeros(max(1, pp.count), dtype=np.uint8)
    lens = np.zeros(max(1, pp.count), dtype=np.uint64)
    _check(_lib.lcs_threshold_batch(ctx.h, pp.ptr(), pp.count, ctypes.byref(al.c),
                                    float(min_percent), _u8p(ok),
                                    lens.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))),
           "lcs_threshold_batch")
    return ok[:pp.count].astype(bool), lens[:pp.count]


class Batch:
    """A resident batch (``lcs_batch_create``): inputs uploaded once, run many times."""

    def __init__(self, ctx: Context, pairs, alphabet="dna", traceback: bool = False,
                 graph: bool = False, words_per_lane: int = 0, ckpt_interval: int = 0,
                 persistent_waves: int = 0, plain: bool = False, strip_rows: int = 0,
                 tb_tiles: int = 0, tb_bands: int = 0, threshold: Optional[float] = None,
                 link_items: int = 0, fill_trace: bool = False, tb_round_kib: int = 0,
                 halves: int = 0):
        self.ctx = ctx
        self._pairs = _Pairs(pairs)
        self.count = self._pairs.count
        self._alpha = _alpha(alphabet)
        self.traceback = traceback
        self.cap = self._pairs.cap
        flags = (LCS_WANT_TRACEBACK if traceback else 0) | (LCS_USE_GRAPH if graph else 0)
        if threshold is not None:
            flags |= LCS_THRESHOLD
        if fill_trace:
            flags |= LCS_FILL_TRACE
        t = _tuning(words_per_lane, ckpt_interval, persistent_waves, plain, strip_rows, tb_tiles,
                    tb_bands, link_items, tb_round_kib, halves)
        h = ctypes.c_void_p()
        _check(_lib.lcs_batch_create(ctx.h, self._pairs.ptr(), self.count,
                                     ctypes.byref(self._alpha.c), flags, ctypes.byref(t),
                                     ctypes.byref(h)), "lcs_batch_create")
        self.h = h
        # inputs are on the device now; host copies are no longer needed
        self._pairs = None
        if threshold is not None:
            self.set_threshold(threshold)

    def set_threshold(self, min_percent: float) -> None:
        _check(_lib.lcs_batch_set_threshold(self.h, float(min_percent)), "lcs_batch_set_threshold")

    def decisions(self) -> Tuple[np.ndarray, np.ndarray]:
        """(pass, lengths) of the last threshold pass, as lcs_threshold_batch."""
        ok = np.zeros(max(1, self.count), dtype=np.uint8)
        lens = np.zeros(max(1, self.count), dtype=np.uint64)
        _check(_lib.lcs_batch_decisions(self.h, _u8p(ok),
                                        lens.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))),
               "lcs_batch_decisions")
        return ok[:self.count].astype(bool), lens[:self.count]

    def run(self) -> None:
        _check(_lib.lcs_batch_run(self.h), "lcs_batch_run")

    def lengths(self) -> np.ndarray:
        out = np.zeros(max(1, self.count), dtype=np.uint64)
        _check(_lib.lcs_batch_lengths(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))),
               "lcs_batch_lengths")
        return out[:self.count]

    def tracebacks(self) -> List[bytes]:
        arena = np.empty(max(1, self.cap), dtype=np.uint8)   # written where read back
        offs = np.zeros(max(1, self.count), dtype=np.uint64)
        lens = np.zeros(max(1, self.count), dtype=np.uint64)
        P64 = ctypes.POINTER(ctypes.c_uint64)
        _check(_lib.lcs_batch_tracebacks(self.h, _u8p(arena), self.cap, offs.ctypes.data_as(P64),
                                         lens.ctypes.data_as(P64)), "lcs_batch_tracebacks")
        return [arena[int(o):int(o) + int(l)].tobytes()
                for o, l in zip(offs[:self.count], lens[:self.count])]

    def clock_mhz(self) -> float:
        """Shader clock (MHz) measured during the last fill launch."""
        v = ctypes.c_double()
        _check(_lib.lcs_batch_clock(self.h, ctypes.byref(v)), "lcs_batch_clock")
        return float(v.value)

    def fill_trace(self) -> np.ndarray:
        """Schedule records of the last pass's fill items (``lcs_batch_fill_trace``;
        the batch must be created with ``fill_trace=True``), as a structured array
        with the fields of ``lcs_fill_item``."""
        n = ctypes.c_uint64()
        _check(_lib.lcs_batch_fill_trace(self.h, None, 0, ctypes.byref(n)), "lcs_batch_fill_trace")
        out = np.zeros(max(1, n.value), dtype=FILL_ITEM)
        _check(_lib.lcs_batch_fill_trace(self.h, out.ctypes.data, n.value, ctypes.byref(n)),
               "lcs_batch_fill_trace")
        return out[:n.value]

    def info(self) -> dict:
        s = lcs_batch_stats()
        _check(_lib.lcs_batch_info(self.h, ctypes.byref(s)), "lcs_batch_info")
        return s.as_dict()

    def time(self, eager: bool = False) -> Tuple[float, float]:
        """(total_ms, fill_ms) of one run from HIP events on the batch's stream;
        fill_ms is -1 for a graph replay (eager=False on a graph batch)."""
        t, f = ctypes.c_float(), ctypes.c_float()
        _check(_lib.lcs_batch_time(self.h, int(eager), ctypes.byref(t), ctypes.byref(f)),
               "lcs_batch_time")
        return float(t.value), float(f.value)

    def close(self) -> None:
        if getattr(self, "h", None):
            _lib.lcs_batch_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The request server (``lcs_server_*``): submit single requests at any
    time; a dispatcher thread in the library batches and runs them."""

    def __init__(self, ctx: Context, mem_budget_bytes: int = 0, streams: int = 0,
                 max_batch_pairs: int = 0):
        self.ctx = ctx
        cfg = lcs_server_config(int(mem_budget_bytes), int(streams), int(max_batch_pairs))
        h = ctypes.c_void_p()
        _check(_lib.lcs_server_create(ctx.h, ctypes.byref(cfg), ctypes.byref(h)), "lcs_server_create")
        self.h = h
        self._alphas = {}
        self._cap = {}

    def submit(self, x, y, alphabet="dna", traceback: bool = False) -> int:
        xa, ya = _as_u8(x), _as_u8(y)
        key = alphabet if isinstance(alphabet, (str, bytes)) else id(alphabet)
        al = self._alphas.get(key)
        if al is None:
            al = self._alphas[key] = _alpha(alphabet)
        t = ctypes.c_uint64(0)
        _check(_lib.lcs_submit(self.h, _u8p(xa), xa.size, _u8p(ya), ya.size, ctypes.byref(al.c),
                               int(bool(traceback)), ctypes.byref(t)), "lcs_submit")
        self._cap[t.value] = (bool(traceback), min(xa.size, ya.size) if traceback else 0)
        return t.value

    def poll(self, ticket: int) -> int:
        return int(_lib.lcs_poll(self.h, ticket))

    def wait(self, ticket: int, timeout_us: int = -1) -> int:
        return int(_lib.lcs_wait(self.h, ticket, int(timeout_us)))

    def result(self, ticket: int):
        """(length, LCS bytes or None, latency in ns) of a finished request."""
        tb, cap = self._cap.get(ticket, (False, 0))
        buf = np.empty(max(cap, 1), dtype=np.uint8)
        L = ctypes.c_uint64(0)
        lat = ctypes.c_uint64(0)
        st = int(_lib.lcs_result(self.h, ticket, ctypes.byref(L), _u8p(buf), cap, ctypes.byref(lat)))
        if st == LCS_PENDING:
            raise LcsError(st, "lcs_result")
        self._cap.pop(ticket, None)
        _check(st, "lcs_result")
        s = buf[: L.value].tobytes() if tb else None
        return int(L.value), s, int(lat.value)

    def cancel(self, ticket: int) -> int:
        return int(_lib.lcs_cancel(self.h, ticket))

    def stats(self) -> dict:
        st = lcs_server_stats()
        _check(_lib.lcs_server_stats_get(self.h, ctypes.byref(st)), "lcs_server_stats_get")
        return st.as_dict()

    def close(self) -> None:
        if getattr(self, "h", None):
            _lib.lcs_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(ctx: Context, pairs, alphabet="dna", traceback: bool = False,
             graph: bool = False) -> Tuple[dict, float]:
    """Timed search for a batch's tuning (``lcs_autotune``); returns the
    tuning fields as a dict (usable as ``Batch(**tuning)``) and its pass time
    in ms."""
    pp = _Pairs(pairs)
    al = _alpha(alphabet)
    flags = (LCS_WANT_TRACEBACK if traceback else 0) | (LCS_USE_GRAPH if graph else 0)
    t = lcs_tuning()
    ms = ctypes.c_float(0.0)
    _check(_lib.lcs_autotune(ctx.h, pp.ptr(), pp.count, ctypes.byref(al.c), flags, ctypes.byref(t),
                             ctypes.byref(ms)), "lcs_autotune")
    return {k: int(getattr(t, k)) for k, _ in lcs_tuning._fields_ if k != "plain"}, float(ms.value)


def plan_describe(m, n, alphabet_size: int = 4, traceback: bool = False, **tuning) -> dict:
    """Host-only: how a batch of these shapes would be packed (no device)."""
    ma = np.ascontiguousarray(np.asarray(m, dtype=np.uint64))
    na = np.ascontiguousarray(np.asarray(n, dtype=np.uint64))
    s = lcs_batch_stats()
    t = _tuning(**tuning)
    P64 = ctypes.POINTER(ctypes.c_uint64)
    _check(_lib.lcs_plan_describe(ma.ctypes.data_as(P64), na.ctypes.data_as(P64), ma.size,
                                  alphabet_size, LCS_WANT_TRACEBACK if traceback else 0,
                                  ctypes.byref(t), ctypes.byref(s)), "lcs_plan_describe")
    return s.as_dict()


def plan_selfcheck(m, n, alphabet_size: int = 4, traceback: bool = False, **tuning) -> int:
    """Host-only structural check of the packer; returns the status code."""
    ma = np.ascontiguousarray(np.asarray(m, dtype=np.uint64))
    na = np.ascontiguousarray(np.asarray(n, dtype=np.uint64))
    t = _tuning(**tuning)
    P64 = ctypes.POINTER(ctypes.c_uint64)
    return int(_lib.lcs_plan_selfcheck(ma.ctypes.data_as(P64), na.ctypes.data_as(P64), ma.size,
                                       alphabet_size, LCS_WANT_TRACEBACK if traceback else 0,
                                       ctypes.byref(t)))
