"""Write the full-size expected values of the benchmark workloads.

Every value here comes from the CPU oracle (``oracle/``) run on the seeded
inputs of ``paper_1306_4627_amd/inputs.py``; nothing is read from the GPU
library.  The values are the ones the paper defines: the length c[m][n] of
section I.C (procedure LCS-length) and the canonical string of section I.D
(procedure Print-LCS, ties going up), stored as its SHA-256 digest.

Each file starts with a digest of its inputs (SHA-256 over, per pair, the
8-byte little-endian length of X, X, the length of Y and Y), so a test can
tell a change of the input generator from a wrong result.

Usage (CPU only; the 262144-symbol pair and the 4096-pair batch take the
oracle tens of minutes):

    python tests/golden/make_goldens.py [--threads N] [names...]

names: pair_dna_4096 pair_long_related batch_short batch_related serve_set
(default: all).
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1306_4627_amd import inputs  # noqa: E402

# Full c and b tables up to this many cells (5 bytes per cell); above it the
# checkpointed-row oracle (same recurrence and walk, rows stored every R).
FULL_TABLE_CELLS = 200_000_000
CKPT_ROWS = 256


def input_digest(pairs) -> str:
    h = hashlib.sha256()
    for x, y in pairs:
        xb, yb = bytes(x), bytes(y)
        h.update(len(xb).to_bytes(8, "little"))
        h.update(xb)
        h.update(len(yb).to_bytes(8, "little"))
        h.update(yb)
    return h.hexdigest()


def canonical(x, y) -> bytes:
    if len(x) * len(y) <= FULL_TABLE_CELLS:
        return oracle.lcs_traceback(x, y)
    return oracle.lcs_traceback_ckpt(x, y, CKPT_ROWS)


def _header(f, what: str, digest: str):
    f.write(f"# {what}\n")
    f.write("# Expected values from the CPU oracle: length = c[m][n] of paper section I.C\n")
    f.write("# (procedure LCS-length); string = the canonical LCS of section I.D (Print-LCS,\n")
    f.write("# mismatch ties going up), as its SHA-256 digest.\n")
    f.write("# Written by tests/golden/make_goldens.py (calls only oracle/ and the seeded\n")
    f.write("# generators of paper_1306_4627_amd/inputs.py).\n")
    f.write(f"input_sha256 {digest}\n")


def _progress(name: str, done: int, total: int, t0: float):
    print(f"[{name}] {done}/{total} ({time.time() - t0:.0f} s)", flush=True)


def make_pair(name: str, p, threads: int):
    t0 = time.time()
    x, y = p.x, p.y
    s = canonical(x, y)
    L = oracle.lcs_length(x, y)
    assert L == len(s), "oracle length and string disagree"
    path = os.path.join(HERE, f"full_{name}.txt")
    with open(path, "w") as f:
        _header(f, f"workload {name}: one pair, m={x.size}, n={y.size}",
                input_digest([(x, y)]))
        f.write(f"m {x.size}\nn {y.size}\nlength {L}\n")
        f.write(f"string_sha256 {hashlib.sha256(s).hexdigest()}\n")
    print(f"[{name}] L={L} ({time.time() - t0:.0f} s) -> {path}", flush=True)


def make_batch_short(threads: int):
    t0 = time.time()
    pairs = inputs.batch_short()
    xy = [(p.x, p.y) for p in pairs]
    with ThreadPoolExecutor(threads) as ex:
        lens = list(ex.map(lambda q: oracle.lcs_length(q[0], q[1]), xy))
    path = os.path.join(HERE, "full_batch_short.txt")
    with open(path, "w") as f:
        _header(f, f"workload batch_short: {len(pairs)} pairs, lengths only "
                   "(32 per line, input order)", input_digest(xy))
        f.write(f"pairs {len(pairs)}\n")
        for k in range(0, len(lens), 32):
            f.write(" ".join(str(v) for v in lens[k:k + 32]) + "\n")
    print(f"[batch_short] {len(pairs)} lengths ({time.time() - t0:.0f} s) -> {path}", flush=True)


def make_batch_related(threads: int):
    t0 = time.time()
    pairs = inputs.batch_related()
    xy = [(p.x, p.y) for p in pairs]
    order = sorted(range(len(xy)), key=lambda k: -xy[k][0].size * xy[k][1].size)
    res = [None] * len(xy)
    done = [0]

    def one(k):
        x, y = xy[k]
        s = canonical(x, y)
        res[k] = (len(s), hashlib.sha256(s).hexdigest()[:32])
        done[0] += 1
        if done[0] % 256 == 0:
            _progress("batch_related", done[0], len(xy), t0)

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(one, order))
    path = os.path.join(HERE, "full_batch_related.txt")
    with open(path, "w") as f:
        _header(f, f"workload batch_related: {len(pairs)} pairs with tracebacks; per line: "
                   "index m n length first-32-hex-of-string-sha256", input_digest(xy))
        f.write(f"pairs {len(pairs)}\n")
        for k, (x, y) in enumerate(xy):
            f.write(f"{k} {x.size} {y.size} {res[k][0]} {res[k][1]}\n")
    print(f"[batch_related] ({time.time() - t0:.0f} s) -> {path}", flush=True)


def make_serve_set(threads: int):
    t0 = time.time()
    reqs = inputs.serve_set()
    xy = [(r.x, r.y) for r in reqs]

    def one(r):
        if r.want_traceback:
            s = canonical(r.x, r.y)
            return len(s), hashlib.sha256(s).hexdigest()
        return oracle.lcs_length(r.x, r.y), "-"

    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(one, reqs))
    path = os.path.join(HERE, "full_serve_set.txt")
    with open(path, "w") as f:
        _header(f, f"serving-scale request set: {len(reqs)} requests; per line: index alphabet "
                   "m n traceback length string-sha256 (- without traceback)", input_digest(xy))
        f.write(f"requests {len(reqs)}\n")
        for k, r in enumerate(reqs):
            f.write(f"{k} {r.alphabet} {r.x.size} {r.y.size} {int(r.want_traceback)} "
                    f"{res[k][0]} {res[k][1]}\n")
    print(f"[serve_set] ({time.time() - t0:.0f} s) -> {path}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=max(1, (os.cpu_count() or 2) - 1))
    ap.add_argument("names", nargs="*")
    a = ap.parse_args()
    names = a.names or ["pair_dna_4096", "batch_short", "serve_set", "pair_long_related",
                        "batch_related"]
    oracle.build_oracle(force=False)
    for nm in names:
        if nm == "pair_dna_4096":
            make_pair(nm, inputs.pair_dna_4096(), a.threads)
        elif nm == "pair_long_related":
            make_pair(nm, inputs.pair_long_related(), a.threads)
        elif nm == "batch_short":
            make_batch_short(a.threads)
        elif nm == "batch_related":
            make_batch_related(a.threads)
        elif nm == "serve_set":
            make_serve_set(a.threads)
        else:
            raise SystemExit(f"unknown workload {nm}")


if __name__ == "__main__":
    main()
