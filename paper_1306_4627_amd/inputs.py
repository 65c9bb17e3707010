"""Seeded synthetic inputs for the LCS library, its tests and its benchmark.

This module only draws sequences; it holds none of the LCS arithmetic, so the
GPU path and the CPU oracle can both be fed from it without sharing any part
of the method.

Workloads (all synthetic; the paper publishes no input strings, only the
shapes of its DNA parent/child experiments in Table-1):

* ``pair_dna_4096``      one unrelated DNA pair, 4096 x 4096.
* ``pair_long_related``  X of 262144 DNA symbols, Y = X mutated at rate 10%.
* ``batch_short``        65536 unrelated pairs, lengths U{64..1024}, 20 letters.
* ``batch_related``      4096 related DNA pairs, |X| log-uniform in
                         [256, 65536], Y = X mutated at rate U[5%, 30%].
* ``serve_stream``       Poisson request stream, lengths log-uniform in
                         [100, 100000], alphabet per request.

Mutation model (each position of X independently, with probability r):
substitution by one of the other sigma-1 symbols, insertion of a uniform
symbol after it, or deletion; the three kinds are equally likely.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

BASE_SEED = 13064627

DNA = b"ACGT"
PROTEIN = b"ACDEFGHIKLMNPQRSTVWY"
BYTE = bytes(range(256))
ALPHABETS: Dict[str, bytes] = {"dna": DNA, "protein": PROTEIN, "byte": BYTE}


def rng(offset: int, base: int = BASE_SEED) -> np.random.Generator:
    """numpy PCG64 generator seeded with base + offset."""
    return np.random.Generator(np.random.PCG64(base + offset))


def random_seq(g: np.random.Generator, length: int, alphabet: bytes) -> np.ndarray:
    """iid uniform symbols over ``alphabet`` (uint8 array)."""
    a = np.frombuffer(alphabet, dtype=np.uint8)
    return a[g.integers(0, a.size, size=int(length))]


@dataclass
class MutationLog:
    substitutions: int = 0
    insertions: int = 0
    deletions: int = 0


def mutate(g: np.random.Generator, x: np.ndarray, rate: float,
           alphabet: bytes) -> Tuple[np.ndarray, MutationLog]:
    """Apply the substitution / insertion / deletion model to ``x``."""
    a = np.frombuffer(alphabet, dtype=np.uint8)
    sigma = a.size
    x = np.asarray(x, dtype=np.uint8)
    m = x.size
    hit = g.random(m) < rate
    kind = g.integers(0, 3, size=m)          # 0 sub, 1 ins, 2 del
    draw = g.integers(0, max(1, sigma - 1), size=m)
    ins_sym = a[g.integers(0, sigma, size=m)]
    # position of each x symbol within the alphabet
    lut = np.full(256, -1, dtype=np.int64)
    lut[a] = np.arange(sigma)
    code = lut[x]
    sub = hit & (kind == 0)
    ins = hit & (kind == 1)
    dele = hit & (kind == 2)
    y_main = x.copy()
    if sigma > 1 and sub.any():
        # one of the other sigma-1 symbols: skip over the current one
        other = draw[sub] + (draw[sub] >= code[sub])
        y_main[sub] = a[other]
    keep = ~dele
    counts = keep.astype(np.int64) + ins.astype(np.int64)
    out = np.empty(int(counts.sum()), dtype=np.uint8)
    ends = np.cumsum(counts)
    starts = ends - counts
    kpos = starts[keep]
    out[kpos] = y_main[keep]
    ipos = starts[ins] + keep[ins].astype(np.int64)
    out[ipos] = ins_sym[ins]
    log = MutationLog(int(sub.sum()) if sigma > 1 else 0, int(ins.sum()), int(dele.sum()))
    return out, log


@dataclass
class Pair:
    x: np.ndarray
    y: np.ndarray
    alphabet: str = "dna"
    log: Optional[MutationLog] = None

    @property
    def cells(self) -> int:
        return int(self.x.size) * int(self.y.size)


def pair_dna_4096(m: int = 4096, n: int = 4096) -> Pair:
    """One unrelated DNA pair (seeds base+11, base+12)."""
    return Pair(random_seq(rng(11), m, DNA), random_seq(rng(12), n, DNA), "dna")


def pair_long_related(m: int = 262144, rate: float = 0.10) -> Pair:
    """X iid DNA (seed base+21); Y = mutate(X, rate) (seed base+22)."""
    x = random_seq(rng(21), m, DNA)
    y, log = mutate(rng(22), x, rate, DNA)
    return Pair(x, y, "dna", log)


def batch_short(count: int = 65536, lo: int = 64, hi: int = 1024) -> List[Pair]:
    """Unrelated protein pairs with |X|, |Y| independent U{lo..hi}
    (lengths seed base+31, symbols seed base+32)."""
    gl = rng(31)
    lx = gl.integers(lo, hi + 1, size=count)
    ly = gl.integers(lo, hi + 1, size=count)
    gs = rng(32)
    total = int(lx.sum() + ly.sum())
    pool = random_seq(gs, total, PROTEIN)
    out, p = [], 0
    for a, b in zip(lx, ly):
        x = pool[p:p + a]; p += a
        y = pool[p:p + b]; p += b
        out.append(Pair(x, y, "protein"))
    return out


def batch_related(count: int = 4096, lo: int = 256, hi: int = 65536,
                  rlo: float = 0.05, rhi: float = 0.30) -> List[Pair]:
    """Related DNA pairs: |X| = floor(exp U(ln lo, ln hi)) (seed base+41),
    X iid DNA (seed base+42), rate ~ U[rlo, rhi] and Y = mutate(X, rate)
    (seed base+43)."""
    gl = rng(41)
    lx = np.floor(np.exp(gl.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)
    lx = np.clip(lx, lo, hi)
    gx = rng(42)
    gm = rng(43)
    rates = gm.uniform(rlo, rhi, size=count)
    out = []
    for a, r in zip(lx, rates):
        x = random_seq(gx, int(a), DNA)
        y, log = mutate(gm, x, float(r), DNA)
        out.append(Pair(x, y, "dna", log))
    return out


@dataclass
class Request:
    arrival_s: float
    x: np.ndarray
    y: np.ndarray
    alphabet: str
    want_traceback: bool


def serve_stream(rate_hz: float, count: int, seed_offset: int = 51,
                 lo: int = 100, hi: int = 100000) -> List[Request]:
    """Poisson arrivals at ``rate_hz``; |X| and |Y| independent log-uniform in
    [lo, hi]; alphabet uniform over dna/protein/byte; traceback with
    probability 1/2."""
    g = rng(seed_offset)
    gaps = g.exponential(1.0 / rate_hz, size=count)
    t = np.cumsum(gaps)
    names = ["dna", "protein", "byte"]
    out = []
    for k in range(count):
        lx = int(np.floor(np.exp(g.uniform(np.log(lo), np.log(hi)))))
        ly = int(np.floor(np.exp(g.uniform(np.log(lo), np.log(hi)))))
        al = names[int(g.integers(0, 3))]
        x = random_seq(g, lx, ALPHABETS[al])
        y = random_seq(g, ly, ALPHABETS[al])
        out.append(Request(float(t[k]), x, y, al, bool(g.integers(0, 2))))
    return out


def serve_set(count: int = 24, seed_offset: int = 61, lo: int = 10000,
              hi: int = 100000) -> List[Request]:
    """A fixed set of serving-scale requests (arrival times 0): |X| and |Y|
    log-uniform in [lo, hi], alphabets cycling dna/protein/byte, traceback
    for every other request; every third request is related (Y = X mutated
    at a rate in [5%, 30%]), the others unrelated (independent Y)."""
    g = rng(seed_offset)
    names = ["dna", "protein", "byte"]
    out = []
    for k in range(count):
        al = names[k % 3]
        lx = int(np.floor(np.exp(g.uniform(np.log(lo), np.log(hi)))))
        x = random_seq(g, lx, ALPHABETS[al])
        if k % 3 == 1:
            y, _ = mutate(g, x, float(g.uniform(0.05, 0.30)), ALPHABETS[al])
        else:
            ly = int(np.floor(np.exp(g.uniform(np.log(lo), np.log(hi)))))
            y = random_seq(g, ly, ALPHABETS[al])
        out.append(Request(0.0, x, y, al, k % 2 == 0))
    return out
