"""Tracebacks in rounds (bounded history) against the oracle, bit-exact.

In rounds the fill stores only lengths and the carry words handed between
the work items of long pairs; the items are then refilled a few at a time,
top of each pair first, and each round walks the strips its items hold from
where the previous round's walk left the path.  The strings must be the
canonical ones whatever the round size, including one work item per round.
"""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import golden_data as gd
import oracle
from paper_1306_4627_amd import inputs

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


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


def _canonical(pairs):
    def one(p):
        x, y = p
        if (len(x) + 1) * (len(y) + 1) > 2e8:
            return oracle.lcs_traceback_ckpt(x, y, 512)
        return oracle.lcs_traceback(x, y)
    with ThreadPoolExecutor(THREADS) as ex:
        return list(ex.map(one, pairs))


def _mixed(seed, count, lo, hi, alphabet):
    g = inputs.rng(seed)
    out = []
    for k in range(count):
        m = int(np.exp(g.uniform(np.log(lo), np.log(hi))))
        x = inputs.random_seq(g, m, alphabet)
        if k % 3:
            y, _ = inputs.mutate(g, x, float(g.uniform(0.05, 0.3)), alphabet)
        else:
            y = inputs.random_seq(g, int(np.exp(g.uniform(np.log(lo), np.log(hi)))), alphabet)
        out.append((x, y))
    return out


@pytest.mark.parametrize("wpl", [1, 2])
def test_rounds_of_one_item_and_more(ctx, lcs, wpl):
    # chains of up to 5 items, pairs sharing items, unrelated pairs whose
    # walks leave strips far from the straight line
    pairs = _mixed(9100 + wpl, 40, 30, 18000 * wpl, inputs.DNA)
    pairs += [(inputs.random_seq(inputs.rng(9110), 1, inputs.DNA), inputs.random_seq(inputs.rng(9111), 9, inputs.DNA))]
    want = _canonical(pairs)
    full = lcs.plan_describe([len(x) for x, _ in pairs], [len(y) for _, y in pairs], 4,
                             traceback=True, words_per_lane=wpl)
    shape = ([len(x) for x, _ in pairs], [len(y) for _, y in pairs])
    # the smallest round sizes that hold the largest item, and one larger
    sizes = []
    for kib in (64, 128, 256, 384, 512, 768, 1024, 1536, 2048):
        try:
            d = lcs.plan_describe(*shape, 4, traceback=True, words_per_lane=wpl, tb_round_kib=kib)
        except lcs.LcsError as e:
            assert e.status == lcs.LCS_ERR_NOMEM
            continue
        if d["tb_rounds"] >= 2:
            sizes.append((kib, d))
    assert len(sizes) >= 2
    # below one item's history: refused before any launch
    _say(f"rounds wpl={wpl} 1 KiB: refused")
    with pytest.raises(lcs.LcsError) as e:
        lcs.Batch(ctx, pairs, "dna", traceback=True, words_per_lane=wpl, tb_round_kib=1)
    assert e.value.status == lcs.LCS_ERR_NOMEM
    for kib, d in (sizes[0], sizes[-1]):
        assert d["history_bytes"] < full["history_bytes"]
        assert lcs.plan_selfcheck(*shape, 4, traceback=True, words_per_lane=wpl, tb_round_kib=kib) == 0
        _say(f"rounds wpl={wpl} {kib} KiB: {d['tb_rounds']} rounds")
        with lcs.Batch(ctx, pairs, "dna", traceback=True, graph=True, words_per_lane=wpl,
                       tb_round_kib=kib) as b:
            info = b.info()
            assert info["tb_rounds"] == d["tb_rounds"]
            for rep in range(2):
                b.run()
                assert b.tracebacks() == want, f"{kib} KiB replay {rep}"
                assert list(b.lengths()) == [len(s) for s in want]


def test_rounds_one_item_each_long_chain(ctx, lcs):
    # the smallest rounds: one work item per round, a 40000-row related pair
    # (ten items at one word per lane) and its unrelated counterpart
    x = inputs.random_seq(inputs.rng(21), 40000, inputs.DNA)
    y, _ = inputs.mutate(inputs.rng(22), x, 0.10, inputs.DNA)
    z = inputs.random_seq(inputs.rng(23), 41000, inputs.DNA)
    pairs = [(x, y), (z, x)]
    want = _canonical(pairs)
    # KiB of the largest item's history at one word per lane (16 bytes per
    # step; the steps are the columns plus the lane skew, under 2048 here)
    per_item = 16 * (max(len(y), len(x)) + 2048) // 1024
    _say(f"rounds of one item, {per_item} KiB")
    with lcs.Batch(ctx, pairs, "dna", traceback=True, words_per_lane=1, tb_round_kib=per_item) as b:
        assert b.info()["tb_rounds"] >= 10
        b.run()
        assert b.tracebacks() == want


def test_rounds_chosen_by_the_budget(ctx, lcs):
    # a context whose budget cannot hold the full history: the batch plans
    # rounds by itself, and the one-call entry points work in it
    pairs = _mixed(9200, 12, 2000, 40000, inputs.DNA)
    want = _canonical(pairs)
    shape = ([len(x) for x, _ in pairs], [len(y) for _, y in pairs])
    full = lcs.plan_describe(*shape, 4, traceback=True)
    budget = int(full["history_bytes"] // 3) + (2 << 20)
    small = lcs.Context(0, mem_budget_bytes=budget)
    try:
        _say(f"rounds by budget ({budget >> 20} MiB, full history {full['history_bytes'] >> 20} MiB)")
        with lcs.Batch(small, pairs, "dna", traceback=True) as b:
            info = b.info()
            assert info["tb_rounds"] >= 2 and info["device_bytes"] <= budget
            b.run()
            assert b.tracebacks() == want
        assert lcs.lcs_traceback_batch(small, pairs, "dna") == want
        x, y = pairs[int(np.argmax([len(a) * len(b) for a, b in pairs]))]
        assert lcs.lcs_traceback(small, x, y, "dna") == oracle.lcs_traceback_ckpt(x, y, 512)
    finally:
        small.close()


def test_rounds_edge_lengths(ctx, lcs):
    g = inputs.rng(9300)
    lens = [0, 1, 63, 64, 65, 4095, 4096, 4097, 8191, 8192, 8193, 12289]
    pairs = [(inputs.random_seq(g, m, b"AB"), inputs.random_seq(g, n, b"AB"))
             for m in lens for n in (0, 1, 64, 700)]
    want = _canonical(pairs)
    _say("rounds edge lengths")
    with lcs.Batch(ctx, pairs, b"AB", traceback=True, words_per_lane=1, tb_round_kib=64) as b:
        assert b.info()["tb_rounds"] >= 2
        b.run()
        assert b.tracebacks() == want


def test_server_request_runs_in_rounds_when_its_history_exceeds_the_arena(ctx, lcs):
    # a request whose full history does not fit the server's arena (but
    # whose inputs and one item's history do) completes in rounds
    g = inputs.rng(9400)
    x = inputs.random_seq(g, 30000, inputs.DNA)
    y, _ = inputs.mutate(g, x, 0.2, inputs.DNA)
    small = (inputs.random_seq(g, 700, inputs.DNA), inputs.random_seq(g, 650, inputs.DNA))
    want = oracle.lcs_traceback_ckpt(x, y, 512)
    full = lcs.plan_describe([x.size], [y.size], 4, traceback=True)
    arena = 3 << 20
    assert full["history_bytes"] > arena
    _say("server request in rounds")
    with lcs.Server(ctx, mem_budget_bytes=arena) as srv:
        t = srv.submit(x, y, "dna", traceback=True)
        ts = srv.submit(*small, "dna", traceback=True)
        assert srv.wait(t, 60_000_000) == 0
        assert srv.wait(ts, 60_000_000) == 0
        L, s, _ = srv.result(t)
        assert s == want and L == len(want)
        assert srv.result(ts)[1] == oracle.lcs_traceback(*small)
        assert srv.stats()["arena_peak_bytes"] <= arena


@pytest.mark.skipif(not gd.exists("full_pair_long_related.txt"), reason="golden not written")
def test_full_long_related_pair_in_rounds(ctx, lcs):
    # the 262144-row related pair with the history of about 64 MiB at a time
    p = inputs.pair_long_related()
    g = gd.pair("pair_long_related")
    _say("full long related pair in rounds (64 MiB)")
    with lcs.Batch(ctx, [(p.x, p.y)], "dna", traceback=True, words_per_lane=1,
                   tb_round_kib=64 * 1024) as b:
        info = b.info()
        assert info["tb_rounds"] >= 4 and info["history_bytes"] <= 64 << 20
        b.run()
        assert b.lengths()[0] == g.length
        assert gd.string_digest(b.tracebacks()[0]) == g.string_sha256


@pytest.mark.skipif(not gd.exists("full_batch_related.txt"), reason="golden not written")
def test_full_batch_related_in_rounds(ctx, lcs):
    # the 4096-pair related batch with 512 MiB of history at a time
    ps = inputs.batch_related()
    pairs = [(p.x, p.y) for p in ps]
    g = gd.batch_related()
    _say("full related batch in rounds (512 MiB)")
    with lcs.Batch(ctx, pairs, "dna", traceback=True, graph=True, tb_round_kib=512 * 1024) as b:
        assert b.info()["tb_rounds"] >= 2
        b.run()
        L = b.lengths()
        S = b.tracebacks()
    assert np.array_equal(L, g.lengths)
    bad = [k for k in range(len(S)) if gd.string_digest(S[k])[:32] != g.sha_prefix[k]]
    assert not bad, f"{len(bad)} strings differ, first {bad[:8]}"
