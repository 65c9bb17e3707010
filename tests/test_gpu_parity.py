"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
element by element, bit-exact for lengths and traceback strings.

Every case prints its name before it touches the GPU so that a failing run
names it.
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


def _oracle_lengths(pairs):
    with ThreadPoolExecutor(THREADS) as ex:
        return np.array(list(ex.map(lambda p: oracle.lcs_length(p[0], p[1]), pairs)), dtype=np.uint64)


def _oracle_tracebacks(pairs, ckpt_rows=None):
    def one(p):
        x, y = p
        if ckpt_rows or (len(x) + 1) * (len(y) + 1) > 3e8:
            return oracle.lcs_traceback_ckpt(x, y, ckpt_rows or 512)
        return oracle.lcs_traceback(x, y)
    with ThreadPoolExecutor(THREADS) as ex:
        return list(ex.map(one, pairs))


def _rand(g, n, al):
    return inputs.random_seq(g, n, al)


EDGE = [0, 1, 2, 3, 31, 32, 33, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 1000, 1023, 1024, 1025]


@pytest.mark.parametrize("alname", ["dna", "protein", "AB", "A"])
def test_single_pairs_edge_lengths(ctx, lcs, alname):
    al = {"dna": inputs.DNA, "protein": inputs.PROTEIN, "AB": b"AB", "A": b"A"}[alname]
    g = inputs.rng(5000 + len(al))
    lens = [0, 1, 2, 63, 64, 65, 128, 129, 700]
    for m in lens:
        for n in (0, 1, 64, 65, 300):
            x, y = _rand(g, m, al), _rand(g, n, al)
            _say(f"single {alname} m={m} n={n}")
            assert lcs.lcs_length(ctx, x, y, al) == oracle.lcs_length(x, y), (m, n)
            assert lcs.lcs_traceback(ctx, x, y, al) == oracle.lcs_traceback(x, y), (m, n)


@pytest.mark.parametrize("sigma,wpl", [(80, 1), (128, 1), (150, 2), (200, 1), (256, 1), (256, 0)])
def test_wide_alphabets(ctx, lcs, sigma, wpl):
    # alphabets past 127 symbols: the stream holds plain codes and the fill
    # runs fewer waves per work-group; the byte order of the alphabet is
    # shuffled so that codes differ from byte values
    g = inputs.rng(6050 + sigma + wpl)
    syms = bytes(int(v) for v in g.permutation(256)[:sigma])
    pairs = []
    for m in (0, 1, 63, 64, 65, 300, 2000, 5000):
        for n in (0, 1, 64, 129, 1500):
            pairs.append((inputs.random_seq(g, m, syms), inputs.random_seq(g, n, syms)))
    for _ in range(6):
        x = inputs.random_seq(g, int(g.integers(100, 9000)), syms)
        y, _ = inputs.mutate(g, x, float(g.uniform(0.05, 0.3)), syms)
        pairs.append((x, y))
    _say(f"wide alphabet sigma={sigma} wpl={wpl} pairs={len(pairs)}")
    al = None if sigma == 256 and wpl == 0 else syms     # None: all 256 bytes in byte order
    with lcs.Batch(ctx, pairs, al, traceback=True, words_per_lane=wpl) as b:
        b.run()
        L = b.lengths()
        S = b.tracebacks()
    assert np.array_equal(L, _oracle_lengths(pairs))
    assert S == _oracle_tracebacks(pairs)
    p0 = pairs[-1]
    assert lcs.lcs_traceback(ctx, p0[0], p0[1], al) == oracle.lcs_traceback(p0[0], p0[1])


@pytest.mark.parametrize("wpl", [1, 2, 4, 8])
def test_batch_edge_lengths_lengths_and_tracebacks(ctx, lcs, wpl):
    g = inputs.rng(6000 + wpl)
    pairs = []
    for m in EDGE:
        for n in (0, 1, 5, 64, 65, 333, 1025):
            pairs.append((_rand(g, m, inputs.DNA), _rand(g, n, inputs.DNA)))
    _say(f"batch edge wpl={wpl} pairs={len(pairs)}")
    with lcs.Batch(ctx, pairs, "dna", traceback=True, words_per_lane=wpl) as b:
        b.run()
        got_L = b.lengths()
        got_S = b.tracebacks()
    assert np.array_equal(got_L, _oracle_lengths(pairs))
    want_S = _oracle_tracebacks(pairs)
    for k, (a, w) in enumerate(zip(got_S, want_S)):
        assert a == w, f"pair {k}: m={len(pairs[k][0])} n={len(pairs[k][1])}"


@pytest.mark.parametrize("ckpt", [64, 128, 256])
def test_traceback_checkpoint_intervals(ctx, lcs, ckpt):
    g = inputs.rng(6100 + ckpt)
    pairs = []
    for _ in range(30):
        m = int(g.integers(1, 3000))
        x = _rand(g, m, inputs.DNA)
        y, _ = inputs.mutate(g, x, float(g.uniform(0.05, 0.4)), inputs.DNA)
        pairs.append((x, y))
    _say(f"ckpt={ckpt}")
    with lcs.Batch(ctx, pairs, "dna", traceback=True, ckpt_interval=ckpt) as b:
        b.run()
        assert b.tracebacks() == _oracle_tracebacks(pairs)


def _strip_cases(g):
    pairs = []
    for _ in range(24):          # related: the straight-line entry guess is close
        m = int(g.integers(1, 6000))
        x = _rand(g, m, inputs.DNA)
        y, _ = inputs.mutate(g, x, float(g.uniform(0.02, 0.4)), inputs.DNA)
        pairs.append((x, y))
    for _ in range(8):           # unrelated, lopsided: guesses far from the path
        m, n = int(g.integers(1, 4000)), int(g.integers(1, 4000))
        pairs.append((_rand(g, m, inputs.DNA), _rand(g, n, inputs.DNA)))
    A = lambda k: np.full(k, ord("A"), np.uint8)
    C = lambda k: np.full(k, ord("C"), np.uint8)
    pairs += [
        (A(3000), A(500)),                                    # walk ends high up
        (A(500), A(3000)),
        (A(2000), C(1500)),                                   # no match at all
        (A(3000), np.concatenate([C(1000), A(40), C(1000)])),  # short diagonal, long climbs
        (np.frombuffer(b"ACGT" * 700, np.uint8), np.frombuffer(b"CGTA" * 650, np.uint8)),
        (_rand(g, 2500, inputs.DNA), _rand(g, 3, inputs.DNA)),
    ]
    return pairs


@pytest.mark.parametrize("strip_rows,wpl", [(64, 1), (128, 2), (192, 1), (512, 2), (1024, 4)])
def test_traceback_strips(ctx, lcs, strip_rows, wpl):
    # the walk of each pair is cut into strips walked from estimated entry
    # columns and then reconciled; the result must not depend on the cut
    g = inputs.rng(6450 + strip_rows + wpl)
    pairs = _strip_cases(g)
    _say(f"strips rows={strip_rows} wpl={wpl} pairs={len(pairs)}")
    with lcs.Batch(ctx, pairs, "dna", traceback=True, words_per_lane=wpl,
                   strip_rows=strip_rows) as b:
        b.run()
        L = b.lengths()
        S = b.tracebacks()
    assert np.array_equal(L, _oracle_lengths(pairs))
    want = _oracle_tracebacks(pairs)
    for k, (a, w) in enumerate(zip(S, want)):
        assert a == w, f"pair {k}: m={len(pairs[k][0])} n={len(pairs[k][1])}"


@pytest.mark.parametrize("tiles", [1, 3, 8])
def test_traceback_strips_plain_and_tiles(ctx, lcs, tiles):
    g = inputs.rng(6470 + tiles)
    pairs = _strip_cases(g)[::3]
    want = _oracle_tracebacks(pairs)
    _say(f"strips plain tiles={tiles} pairs={len(pairs)}")
    with lcs.Batch(ctx, pairs, "dna", traceback=True, plain=True, strip_rows=256,
                   tb_tiles=tiles) as b:
        b.run()
        assert b.tracebacks() == want
    with lcs.Batch(ctx, pairs, "dna", traceback=True, graph=True, strip_rows=128,
                   tb_tiles=tiles) as b:
        for rep in range(2):
            b.run()
            assert b.tracebacks() == want, rep


def test_autotune_picks_a_valid_tuning_and_caches_it(ctx, lcs):
    g = inputs.rng(6490)
    pairs = []
    for _ in range(60):
        m = int(np.exp(g.uniform(np.log(64), np.log(6000))))
        x = _rand(g, m, inputs.DNA)
        y, _ = inputs.mutate(g, x, float(g.uniform(0.05, 0.3)), inputs.DNA)
        pairs.append((x, y))
    _say("autotune")
    tun, ms = lcs.autotune(ctx, pairs, "dna", traceback=True, graph=True)
    assert tun["words_per_lane"] in (1, 2, 4, 8) and ms > 0
    assert tun["ckpt_interval"] in (0, 64, 128, 256)
    import time
    t0 = time.perf_counter()
    tun2, ms2 = lcs.autotune(ctx, pairs, "dna", traceback=True, graph=True)
    assert tun2 == tun and ms2 == ms and time.perf_counter() - t0 < 0.5   # from the cache
    with lcs.Batch(ctx, pairs, "dna", traceback=True, graph=True, **tun) as b:
        b.run()
        assert np.array_equal(b.lengths(), _oracle_lengths(pairs))
        assert b.tracebacks() == _oracle_tracebacks(pairs)
    # lengths only: a different shape key, a words-per-lane search of its own
    tun3, _ = lcs.autotune(ctx, pairs, "dna")
    with lcs.Batch(ctx, pairs, "dna", **tun3) as b:
        b.run()
        assert np.array_equal(b.lengths(), _oracle_lengths(pairs))


@pytest.mark.parametrize("wpl", [1, 2, 4])
def test_chained_items_long_rows(ctx, lcs, wpl):
    # rows beyond one wave (64 lanes * wpl words * 64 bits) chain several
    # work items through memory
    g = inputs.rng(6200 + wpl)
    pairs = []
    for m in (4095, 4096, 4097, 8192 + 1, 64 * 64 * wpl * 2 + 65, 20000):
        x = _rand(g, m, inputs.DNA)
        y, _ = inputs.mutate(g, x, 0.2, inputs.DNA)
        pairs.append((x, y))
        pairs.append((_rand(g, m, inputs.DNA), _rand(g, int(g.integers(1, 5000)), inputs.DNA)))
    _say(f"chains wpl={wpl}")
    with lcs.Batch(ctx, pairs, "dna", traceback=True, words_per_lane=wpl) as b:
        b.run()
        L = b.lengths()
        S = b.tracebacks()
    assert np.array_equal(L, _oracle_lengths(pairs))
    assert S == _oracle_tracebacks(pairs)


def test_adversarial_inputs(ctx, lcs):
    g = inputs.rng(6300)
    x = _rand(g, 5000, inputs.DNA)
    cases = {
        "x_eq_y": (x, x.copy()),
        "all_same": (np.full(3000, ord("A"), np.uint8), np.full(2000, ord("A"), np.uint8)),
        "disjoint": (np.full(3000, ord("A"), np.uint8), np.full(2500, ord("C"), np.uint8)),
        "periodic": (np.frombuffer(b"ACGT" * 1000, np.uint8), np.frombuffer(b"CGTA" * 900, np.uint8)),
        "ripple": (np.full(4100, ord("A"), np.uint8), np.frombuffer(b"A" + b"C" * 3000 + b"A" * 50, np.uint8)),
        "subseq": (x[::3].copy(), x),
        "one_row": (x[:1], x),
        "one_col": (x, x[:1]),
    }
    pairs = list(cases.values())
    _say("adversarial batch")
    for wpl in (1, 4):
        with lcs.Batch(ctx, pairs, "dna", traceback=True, words_per_lane=wpl) as b:
            b.run()
            L = b.lengths()
            S = b.tracebacks()
        for (name, (a, c)), l, s in zip(cases.items(), L, S):
            assert l == oracle.lcs_length(a, c), name
            assert s == oracle.lcs_traceback(a, c), name
    assert S[0] == x.tobytes()


def test_batch_order_and_plain_agree(ctx, lcs):
    g = inputs.rng(6400)
    pairs = []
    for _ in range(300):
        m, n = int(g.integers(0, 2500)), int(g.integers(0, 2500))
        pairs.append((_rand(g, m, inputs.PROTEIN), _rand(g, n, inputs.PROTEIN)))
    _say("order/plain")
    with lcs.Batch(ctx, pairs, "protein", traceback=True) as b:
        b.run()
        L1, S1 = b.lengths(), b.tracebacks()
    perm = g.permutation(len(pairs))
    with lcs.Batch(ctx, [pairs[k] for k in perm], "protein", traceback=True) as b:
        b.run()
        L2, S2 = b.lengths(), b.tracebacks()
    with lcs.Batch(ctx, pairs[:60], "protein", traceback=True, plain=True) as b:
        b.run()
        L3, S3 = b.lengths(), b.tracebacks()
    assert np.array_equal(L1, _oracle_lengths(pairs))
    assert np.array_equal(L2, L1[perm])
    assert [S2[k] for k in range(len(perm))] == [S1[k] for k in perm]
    assert np.array_equal(L3, L1[:60]) and S3 == S1[:60]
    assert S1 == _oracle_tracebacks(pairs)


def test_graph_replays_match_eager(ctx, lcs):
    g = inputs.rng(6500)
    pairs = [(_rand(g, int(a), inputs.DNA), _rand(g, int(c), inputs.DNA))
             for a, c in g.integers(1, 6000, size=(50, 2))]
    want_L = _oracle_lengths(pairs)
    want_S = _oracle_tracebacks(pairs)
    _say("graph replays")
    with lcs.Batch(ctx, pairs, "dna", traceback=True, graph=True) as b:
        for rep in range(4):
            b.run()
            assert np.array_equal(b.lengths(), want_L), rep
            assert b.tracebacks() == want_S, rep
            # eager work between replays
            assert lcs.lcs_length(ctx, pairs[rep][0], pairs[rep][1], "dna") == want_L[rep]


def test_one_call_batch_entry_points(ctx, lcs):
    g = inputs.rng(6600)
    pairs = [(_rand(g, int(a), inputs.PROTEIN), _rand(g, int(c), inputs.PROTEIN))
             for a, c in g.integers(0, 900, size=(100, 2))]
    _say("one-call batch")
    L = lcs.lcs_length_batch(ctx, pairs, "protein")
    S = lcs.lcs_traceback_batch(ctx, pairs, "protein")
    assert np.array_equal(L, _oracle_lengths(pairs))
    assert S == _oracle_tracebacks(pairs)


def test_bit_vector_identity_through_prefixes(ctx, lcs):
    # c[i][n] for every prefix X_i equals the LCS length of (X_i, Y): the
    # batch of all prefixes pins every bit of the final column vector
    g = inputs.rng(6700)
    x = _rand(g, 300, inputs.DNA)
    y = _rand(g, 280, inputs.DNA)
    pairs = [(x[:i], y) for i in range(0, 301)]
    _say("prefix column")
    got = lcs.lcs_length_batch(ctx, pairs, "dna")
    c, _ = oracle.lcs_tables(x, y)
    assert np.array_equal(got, c[:, -1].astype(np.uint64))


def test_error_paths_leave_outputs_untouched(ctx, lcs):
    _say("error paths")
    with pytest.raises(lcs.LcsError) as e:
        lcs.lcs_length(ctx, b"ACGX", b"ACG", "dna")
    assert e.value.status == lcs.LCS_ERR_SYMBOL
    with pytest.raises(lcs.LcsError) as e:
        lcs.Batch(ctx, [(b"AC", b"CA")], "dna", words_per_lane=3)
    assert e.value.status == lcs.LCS_ERR_ARG
    small = lcs.Context(0, mem_budget_bytes=4096)
    with pytest.raises(lcs.LcsError) as e:
        lcs.Batch(small, [(b"ACGT" * 100, b"TGCA" * 100)], "dna")
    assert e.value.status == lcs.LCS_ERR_NOMEM
    small.close()


@pytest.mark.parametrize("where", ["first", "middle", "last"])
def test_symbol_errors_in_large_batches(ctx, lcs, where):
    # a batch large enough that its bytes are validated by several host
    # threads (about 96 MB): one foreign byte in the first, a middle or the
    # last pair is found, and nothing runs
    g = inputs.rng(7400)
    base = _rand(g, 1 << 20, inputs.DNA)
    pairs = [(base, base) for _ in range(48)]
    k = {"first": 0, "middle": 23, "last": 47}[where]
    bad = base.copy()
    bad[len(bad) // 2 + k] = ord("N")
    pairs[k] = (base, bad) if k % 2 else (bad, base)
    _say(f"symbol error in a large batch ({where})")
    with pytest.raises(lcs.LcsError) as e:
        lcs.Batch(ctx, pairs, "dna")
    assert e.value.status == lcs.LCS_ERR_SYMBOL
    with pytest.raises(lcs.LcsError) as e:
        lcs.lcs_length_batch(ctx, pairs, "dna")
    assert e.value.status == lcs.LCS_ERR_SYMBOL


@pytest.mark.parametrize("sigma", [20, 40])
def test_lengths_with_next_item_prefetch(ctx, lcs, sigma):
    # alphabets whose match masks leave two waves or fewer per SIMD at two
    # words per lane: the lengths-only fill prefetches each wave's next item
    # (its ticket, lane tables, X codes and first stream values) during the
    # current one; short pairs packed many per item, single-item pairs and
    # chains of several items, ragged lengths, empty pairs
    g = inputs.rng(8600 + sigma)
    al = bytes(range(65, 65 + sigma))
    pairs = []
    for k in range(300):
        m = int(g.integers(0, 1100)) if k % 10 else int(g.integers(8000, 30000))
        n = int(g.integers(0, 1100)) if k % 7 else int(g.integers(2000, 9000))
        pairs.append((_rand(g, m, al), _rand(g, n, al)))
    want = _oracle_lengths(pairs)
    for wpl in (2, 1):
        _say(f"prefetch fill sigma={sigma} wpl={wpl}")
        with lcs.Batch(ctx, pairs, al, graph=True, words_per_lane=wpl) as b:
            for rep in range(2):
                b.run()
                assert np.array_equal(b.lengths(), want), (wpl, rep)
        assert np.array_equal(lcs.lcs_length_batch(ctx, pairs, al), want)


# --------------------------------------------------------------------------
# full-size workloads, in the launch configuration of the benchmark
# --------------------------------------------------------------------------

def test_full_pair_dna_4096(ctx, lcs):
    p = inputs.pair_dna_4096()
    g = gd.pair("pair_dna_4096")
    assert g.input_sha256 == gd.input_digest([(p.x, p.y)]), "input generator changed"
    _say("full 4096x4096 pair")
    assert lcs.lcs_length(ctx, p.x, p.y, "dna") == g.length
    s = lcs.lcs_traceback(ctx, p.x, p.y, "dna")
    assert (len(s), gd.string_digest(s)) == (g.length, g.string_sha256)


def test_full_batch_short(ctx, lcs):
    # every one of the 65536 lengths against the oracle's (stored)
    ps = inputs.batch_short()
    pairs = [(p.x, p.y) for p in ps]
    g = gd.batch_short()
    assert g.input_sha256 == gd.input_digest(pairs), "input generator changed"
    _say("full short batch (65536 pairs), graph replays")
    with lcs.Batch(ctx, pairs, "protein", graph=True) as b:
        for rep in range(2):
            b.run()
            L = b.lengths()
            bad = np.flatnonzero(L != g.lengths)
            assert bad.size == 0, f"replay {rep}: {bad.size} pairs differ, first {bad[:8]}"


def test_full_batch_short_autotuned(ctx, lcs):
    # the benchmark's launch configuration: the autotuner's choice
    ps = inputs.batch_short()
    pairs = [(p.x, p.y) for p in ps]
    g = gd.batch_short()
    _say("full short batch, autotuned")
    tuning, _ = lcs.autotune(ctx, pairs, "protein", traceback=False, graph=True)
    with lcs.Batch(ctx, pairs, "protein", graph=True, **tuning) as b:
        b.run()
        L = b.lengths()
    assert np.array_equal(L, g.lengths), tuning


@pytest.mark.skipif(not gd.exists("full_batch_related.txt"), reason="golden not written")
def test_full_batch_related(ctx, lcs):
    # every one of the 4096 lengths and strings against the oracle's (stored)
    ps = inputs.batch_related()
    pairs = [(p.x, p.y) for p in ps]
    g = gd.batch_related()
    assert g.input_sha256 == gd.input_digest(pairs), "input generator changed"
    _say("full related batch (4096 pairs, tracebacks), autotuned, graph replays")
    tuning, _ = lcs.autotune(ctx, pairs, "dna", traceback=True, graph=True)
    with lcs.Batch(ctx, pairs, "dna", traceback=True, graph=True, **tuning) as b:
        for rep in range(2):
            b.run()
            L = b.lengths()
            S = b.tracebacks()
            bad = np.flatnonzero(L != g.lengths)
            assert bad.size == 0, f"replay {rep}: {bad.size} lengths differ, first {bad[:8]}"
            bad = [k for k in range(len(S)) if gd.string_digest(S[k])[:32] != g.sha_prefix[k]]
            assert not bad, f"replay {rep}: {len(bad)} strings differ, first {bad[:8]}"


@pytest.mark.parametrize("wpl,alname", [(1, "byte"), (2, "protein")])
def test_unrelated_pairs_walked_by_the_seal(ctx, lcs, wpl, alname):
    # unrelated pairs of several strips (walks from different entries rarely
    # meet, so the seal re-walks most strips), beside a related pair and a
    # short unrelated pair of one strip
    g = inputs.rng(9100 + wpl)
    pairs = []
    shapes = (("dna", 20000, 20000), ("protein", 15000, 18000), ("byte", 12000, 9000), ("dna", 3000, 3500))
    for al, m, n in shapes:
        if alname == "protein" and al == "byte":
            continue
        x = inputs.random_seq(g, m, inputs.ALPHABETS[al])
        y = inputs.random_seq(g, n, inputs.ALPHABETS[al])
        pairs.append((x, y))
    x = inputs.random_seq(g, 16000, inputs.DNA)
    y, _ = inputs.mutate(g, x, 0.1, inputs.DNA)
    pairs.append((x, y))
    want = [oracle.lcs_traceback(x, y) for x, y in pairs]
    _say(f"unrelated pairs walked by the seal, wpl {wpl}")
    with lcs.Batch(ctx, pairs, alname, traceback=True, words_per_lane=wpl, strip_rows=4096) as b:
        for rep in range(2):
            b.run()
            L = b.lengths()
            S = b.tracebacks()
            for k, s in enumerate(want):
                assert S[k] == s and L[k] == len(s), (rep, k)


@pytest.mark.skipif(not gd.exists("full_batch_related.txt"), reason="golden not written")
@pytest.mark.parametrize("waves", [1100, 2100, 3500])
def test_full_batch_related_uneven_first_item_bands(ctx, lcs, waves):
    # persistent grids of one, two and three first-item bands (waves per
    # SIMD rounded down); where the work-groups land unevenly some SIMDs hold
    # fewer waves, their bands' places are left to later waves, and chained
    # items must still find their feeders
    ps = inputs.batch_related()
    pairs = [(p.x, p.y) for p in ps]
    g = gd.batch_related()
    _say(f"full related batch, {waves} persistent waves")
    with lcs.Batch(ctx, pairs, "dna", traceback=True, words_per_lane=2, persistent_waves=waves) as b:
        b.run()
        L = b.lengths()
        S = b.tracebacks()
    bad = np.flatnonzero(L != g.lengths)
    assert bad.size == 0, f"{bad.size} lengths differ, first {bad[:8]}"
    bad = [k for k in range(len(S)) if gd.string_digest(S[k])[:32] != g.sha_prefix[k]]
    assert not bad, f"{len(bad)} strings differ, first {bad[:8]}"


@pytest.mark.skipif(not gd.exists("full_pair_long_related.txt"), reason="golden not written")
def test_full_long_related_pair(ctx, lcs):
    p = inputs.pair_long_related()
    g = gd.pair("pair_long_related")
    assert g.input_sha256 == gd.input_digest([(p.x, p.y)]), "input generator changed"
    _say("full long related pair 262144")
    assert lcs.lcs_length(ctx, p.x, p.y, "dna") == g.length
    S = lcs.lcs_traceback(ctx, p.x, p.y, "dna")
    assert (len(S), gd.string_digest(S)) == (g.length, g.string_sha256)
    # the benchmark's resident batch of this pair, graph replays
    with lcs.Batch(ctx, [(p.x, p.y)], "dna", traceback=True, graph=True, words_per_lane=1) as b:
        for rep in range(2):
            b.run()
            assert b.lengths()[0] == g.length
            s2 = b.tracebacks()[0]
            assert gd.string_digest(s2) == g.string_sha256, f"replay {rep}"


def test_long_related_pair_scaled_exact(ctx, lcs):
    # same recipe and launch shape (chained items) at a size the oracle
    # finishes in seconds
    x = inputs.random_seq(inputs.rng(21), 40000, inputs.DNA)
    y, _ = inputs.mutate(inputs.rng(22), x, 0.10, inputs.DNA)
    _say("long related pair 40000 exact")
    assert lcs.lcs_length(ctx, x, y, "dna") == oracle.lcs_length(x, y)
    assert lcs.lcs_traceback(ctx, x, y, "dna") == oracle.lcs_traceback_ckpt(x, y, 1024)


def test_chains_starting_in_shared_items(ctx, lcs):
    # long pairs whose chains start in the free lanes of the item before
    # them (link_items > 1): lengths and strings exact, lengths-only and
    # threshold passes too
    g = inputs.rng(8400)
    pairs = []
    for k in range(14):
        m = int(g.integers(9000, 9400))
        x = _rand(g, m, inputs.DNA)
        y, _ = inputs.mutate(g, x, float(g.uniform(0.05, 0.25)), inputs.DNA)
        pairs.append((x.tobytes(), y.tobytes()))
    pairs += [(_rand(g, 300, inputs.DNA).tobytes(), _rand(g, 9100, inputs.DNA).tobytes())]
    want_s = _oracle_tracebacks(pairs)
    want_l = np.array([len(s) for s in want_s], dtype=np.uint64)
    d = lcs.plan_describe([len(x) for x, _ in pairs], [len(y) for _, y in pairs], 4,
                          traceback=True, words_per_lane=1, link_items=32)
    d1 = lcs.plan_describe([len(x) for x, _ in pairs], [len(y) for _, y in pairs], 4,
                           traceback=True, words_per_lane=1, link_items=1)
    assert d["groups"] < d1["groups"]       # some chains do share an item
    _say("shared-item chains, traceback")
    with lcs.Batch(ctx, pairs, "dna", traceback=True, words_per_lane=1, link_items=32) as b:
        b.run()
        assert b.tracebacks() == want_s
        assert np.array_equal(b.lengths(), want_l)
    _say("shared-item chains, lengths and threshold")
    with lcs.Batch(ctx, pairs, "dna", words_per_lane=1, link_items=32) as b:
        b.run()
        assert np.array_equal(b.lengths(), want_l)
    m = np.array([len(x) for x, _ in pairs], dtype=np.float64)
    sim = (100.0 * want_l.astype(np.float64)) / m
    for pct in (70.0, 85.0, 95.0):
        with lcs.Batch(ctx, pairs, "dna", words_per_lane=1, link_items=32, threshold=pct) as b:
            b.run()
            ok, lens = b.decisions()
            assert np.array_equal(ok, sim >= pct)
            known = lens != lcs.LCS_LENGTH_UNKNOWN
            assert np.array_equal(lens[known], want_l[known])


def test_fill_clock_is_measured(ctx, lcs):
    # the shader clock read by the fill's first wave over its lifetime
    g = inputs.rng(8500)
    pairs = [(_rand(g, 20000, inputs.DNA).tobytes(), _rand(g, 20000, inputs.DNA).tobytes())
             for _ in range(64)]
    _say("fill clock")
    with lcs.Batch(ctx, pairs, "dna") as b:
        with pytest.raises(lcs.LcsError):
            b.clock_mhz()                     # not run yet
        b.time(eager=True)
        mhz = b.clock_mhz()
    assert 300.0 < mhz < 3000.0, mhz
