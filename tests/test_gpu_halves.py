"""GPU parity of the middle-column split (lengths only): a pair's length from
two fills of half its columns each, X against Y[0, h) and X reversed against
Y[h, n) reversed, combined on the device.  Lengths are compared with the
oracle and with the unsplit fill, pair by pair.

Every case prints its name before it touches the GPU so that a failing run
names it.
"""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_1306_4627_amd import inputs

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)
BYTES = bytes(range(256))


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lcs():
    from paper_1306_4627_amd import lcs as mod
    return mod


@pytest.fixture(scope="module")
def ctx(lcs):
    c = lcs.Context(0)
    yield c
    c.close()


def _oracle_lengths(pairs):
    with ThreadPoolExecutor(THREADS) as ex:
        return np.array(list(ex.map(lambda p: oracle.lcs_length(p[0], p[1]), pairs)), dtype=np.uint64)


def _lengths(lcs, ctx, pairs, alphabet, **tuning):
    with lcs.Batch(ctx, pairs, alphabet, **tuning) as b:
        b.run()
        return b.lengths(), b.info()


SIDES = [0, 1, 2, 3, 7, 8, 9, 31, 63, 64, 65, 127, 128, 129, 200, 511, 1000]


@pytest.mark.parametrize("alname,wpl", [("dna", 1), ("dna", 4), ("protein", 2), ("byte", 1),
                                        ("wide100", 2)])
def test_split_edge_lengths(ctx, lcs, alname, wpl):
    # every pair with n >= 2 split; odd and even n, rows inside one word,
    # at a word boundary and across several; all bytes, and 100 symbols at
    # two words per lane, take the plain-code stream
    al = {"dna": inputs.DNA, "protein": inputs.PROTEIN, "byte": BYTES,
          "wide100": bytes(range(100, 200))}[alname]
    g = inputs.rng(7100 + wpl + len(al))
    pairs = []
    for m in SIDES:
        for n in SIDES:
            if (m * 7 + n) % 3 == 0 or m in (0, 1) or n in (0, 1, 2, 3):
                x = inputs.random_seq(g, m, al)
                if n <= m and (m + n) % 2:
                    y = x[:n]            # Y a prefix of X
                else:
                    y = inputs.random_seq(g, n, al)
                pairs.append((x, y))
    _say(f"split edge lengths {alname} wpl={wpl} ({len(pairs)} pairs)")
    alpha = alname if alname in ("dna", "protein", "byte") else al
    L, info = _lengths(lcs, ctx, pairs, alpha, words_per_lane=wpl, halves=2)
    assert info["split_pairs"] == sum(1 for x, y in pairs if len(x) >= 1 and len(y) >= 2)
    want = _oracle_lengths(pairs)
    bad = [(len(pairs[k][0]), len(pairs[k][1]), int(L[k]), int(want[k]))
           for k in range(len(pairs)) if L[k] != want[k]]
    assert not bad, f"{len(bad)} lengths differ, first {bad[:8]}"
    L1, info1 = _lengths(lcs, ctx, pairs, alpha, words_per_lane=wpl, halves=1)
    assert info1["split_pairs"] == 0
    assert np.array_equal(L, L1)


@pytest.mark.parametrize("wpl", [1, 2, 4])
def test_split_chained_rows(ctx, lcs, wpl):
    # halves of pairs longer than one wave chain several work items, in both
    # halves; related and unrelated Y, Y shorter and longer than X
    g = inputs.rng(7200 + wpl)
    pairs = []
    for m in (4095, 4097, 64 * 64 * wpl * 2 + 65, 20000):
        x = inputs.random_seq(g, m, inputs.DNA)
        y, _ = inputs.mutate(g, x, 0.15, inputs.DNA)
        pairs.append((x, y))
        pairs.append((inputs.random_seq(g, m, inputs.DNA),
                      inputs.random_seq(g, int(g.integers(2, 9000)), inputs.DNA)))
    _say(f"split chained rows wpl={wpl}")
    L, info = _lengths(lcs, ctx, pairs, "dna", words_per_lane=wpl, halves=2)
    assert info["split_pairs"] == len(pairs)
    assert np.array_equal(L, _oracle_lengths(pairs))


def test_split_chosen_automatically(ctx, lcs):
    # a lone long pair is split by default; a batch that fills the device is
    # not, and neither is a traceback batch
    x = inputs.random_seq(inputs.rng(31), 40000, inputs.DNA)
    y, _ = inputs.mutate(inputs.rng(32), x, 0.10, inputs.DNA)
    _say("split automatic: one 40000 related pair")
    want = oracle.lcs_length(x, y)
    L, info = _lengths(lcs, ctx, [(x, y)], "dna")
    assert info["split_pairs"] == 1 and int(L[0]) == want
    assert lcs.lcs_length(ctx, x, y, "dna") == want
    with lcs.Batch(ctx, [(x, y)], "dna", traceback=True) as b:
        assert b.info()["split_pairs"] == 0
    g = inputs.rng(33)
    many = [(inputs.random_seq(g, 4096, inputs.DNA), inputs.random_seq(g, 4096, inputs.DNA))
            for _ in range(600)]
    _say("split automatic: 600 pairs of 4096 (not split)")
    with lcs.Batch(ctx, many, "dna") as b:
        assert b.info()["split_pairs"] == 0


def test_split_graph_replays(ctx, lcs):
    g = inputs.rng(7300)
    pairs = []
    for m, n in ((5000, 7001), (9000, 300), (1, 2), (700, 12001), (64, 64)):
        x = inputs.random_seq(g, m, inputs.PROTEIN)
        y = inputs.mutate(g, x, 0.3, inputs.PROTEIN)[0] if m == n else inputs.random_seq(g, n, inputs.PROTEIN)
        pairs.append((x, y))
    want = _oracle_lengths(pairs)
    _say("split graph replays")
    with lcs.Batch(ctx, pairs, "protein", graph=True, halves=2) as b:
        assert b.info()["split_pairs"] == len(pairs)
        for rep in range(3):
            b.run()
            assert np.array_equal(b.lengths(), want), f"replay {rep}"
