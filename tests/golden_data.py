"""Readers of the full-size expected values in ``tests/golden/full_*.txt``.

The files are written by ``tests/golden/make_goldens.py`` from the CPU oracle
alone (no GPU value is ever stored).  Each starts with a SHA-256 digest of
its inputs, recomputed here from the seeded generators, so a test tells a
changed input generator apart from a wrong result.
"""
from __future__ import annotations

import hashlib
import os
from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def input_digest(pairs) -> str:
    h = hashlib.sha256()
    for x, y in pairs:
        xb, yb = bytes(np.asarray(x, dtype=np.uint8)), bytes(np.asarray(y, dtype=np.uint8))
        h.update(len(xb).to_bytes(8, "little"))
        h.update(xb)
        h.update(len(yb).to_bytes(8, "little"))
        h.update(yb)
    return h.hexdigest()


def string_digest(s: bytes) -> str:
    return hashlib.sha256(bytes(s)).hexdigest()


def _lines(name: str) -> List[str]:
    path = os.path.join(HERE, name)
    with open(path) as f:
        return [ln.rstrip("\n") for ln in f if ln.strip() and not ln.startswith("#")]


def _head(lines: List[str]) -> Dict[str, str]:
    out = {}
    for ln in lines:
        k, _, v = ln.partition(" ")
        out.setdefault(k, v)
    return out


def exists(name: str) -> bool:
    return os.path.exists(os.path.join(HERE, name))


@dataclass
class PairGolden:
    input_sha256: str
    m: int
    n: int
    length: int
    string_sha256: str


def pair(name: str) -> PairGolden:
    h = _head(_lines(f"full_{name}.txt"))
    return PairGolden(h["input_sha256"], int(h["m"]), int(h["n"]), int(h["length"]),
                      h["string_sha256"])


@dataclass
class LengthsGolden:
    input_sha256: str
    lengths: np.ndarray


def batch_short() -> LengthsGolden:
    lines = _lines("full_batch_short.txt")
    h = _head(lines)
    count = int(h["pairs"])
    vals = []
    for ln in lines:
        if ln.startswith(("input_sha256", "pairs")):
            continue
        vals.extend(int(v) for v in ln.split())
    assert len(vals) == count, "truncated golden file"
    return LengthsGolden(h["input_sha256"], np.array(vals, dtype=np.uint64))


@dataclass
class BatchGolden:
    input_sha256: str
    m: np.ndarray
    n: np.ndarray
    lengths: np.ndarray
    sha_prefix: List[str]     # first 32 hex digits of each string's SHA-256


def batch_related() -> BatchGolden:
    lines = _lines("full_batch_related.txt")
    h = _head(lines)
    count = int(h["pairs"])
    m, n, L, sh = [], [], [], []
    for ln in lines:
        if ln.startswith(("input_sha256", "pairs")):
            continue
        k, a, b, l, s = ln.split()
        assert int(k) == len(m)
        m.append(int(a))
        n.append(int(b))
        L.append(int(l))
        sh.append(s)
    assert len(m) == count, "truncated golden file"
    return BatchGolden(h["input_sha256"], np.array(m), np.array(n), np.array(L, dtype=np.uint64), sh)


@dataclass
class RequestGolden:
    alphabet: str
    m: int
    n: int
    traceback: bool
    length: int
    string_sha256: Optional[str]


def serve_set():
    lines = _lines("full_serve_set.txt")
    h = _head(lines)
    count = int(h["requests"])
    out = []
    for ln in lines:
        if ln.startswith(("input_sha256", "requests")):
            continue
        k, al, m, n, tb, l, s = ln.split()
        assert int(k) == len(out)
        out.append(RequestGolden(al, int(m), int(n), tb == "1", int(l), None if s == "-" else s))
    assert len(out) == count, "truncated golden file"
    return h["input_sha256"], out
