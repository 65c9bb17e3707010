"""Section II's derived outputs on the GPU against the oracle: the similarity
percentage (bit-exact doubles) and the threshold pass (every yes/no answer
exact, every reported length exact, early stops actually taken), over packed
small pairs, single-wave pairs and chained long pairs, graph replays, the
plain per-pair path, edge cases and the 4096-pair related workload."""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_1306_4627_amd import inputs

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)
UNKNOWN = (1 << 64) - 1


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


def _similarity(pairs):
    with ThreadPoolExecutor(THREADS) as ex:
        return np.array(list(ex.map(lambda p: oracle.similarity_percent(p[0], p[1]), pairs)))


def _lengths(pairs):
    with ThreadPoolExecutor(THREADS) as ex:
        return np.array(list(ex.map(lambda p: oracle.lcs_length(p[0], p[1]), pairs)), dtype=np.uint64)


def _mixed(seed):
    """Small pairs (many per wave), single-wave pairs and chained pairs,
    related at various rates and unrelated."""
    g = inputs.rng(seed)
    pairs = []
    sizes = [int(np.exp(g.uniform(np.log(8), np.log(3000)))) for _ in range(70)]
    sizes += [5000, 8191, 8193, 12000, 20000, 41000]
    for k, m in enumerate(sizes):
        x = inputs.random_seq(g, m, inputs.DNA)
        if k % 3 == 2:
            y = inputs.random_seq(g, int(m * g.uniform(0.5, 1.5)), inputs.DNA)
        else:
            y, _ = inputs.mutate(g, x, float(g.uniform(0.01, 0.35)), inputs.DNA)
        pairs.append((x.tobytes(), y.tobytes()))
    return pairs


@pytest.fixture(scope="module")
def mixed():
    pairs = _mixed(8100)
    return pairs, _similarity(pairs), _lengths(pairs)


def _check(pairs, sim, L, pct, ok, lens):
    want = sim >= pct
    bad = np.nonzero(ok != want)[0]
    assert bad.size == 0, [(int(k), len(pairs[k][0]), len(pairs[k][1]), sim[k]) for k in bad[:5]]
    known = lens != UNKNOWN
    assert np.array_equal(lens[known], L[known])


@pytest.mark.parametrize("wpl", [0, 1, 4])
def test_threshold_answers_match_oracle(ctx, lcs, mixed, wpl):
    pairs, sim, L = mixed
    early = 0
    with lcs.Batch(ctx, pairs, "dna", threshold=50.0, words_per_lane=wpl) as b:
        for pct in [0.0, 30.0, 60.0, 75.0, 85.0, 90.0, 95.0, 99.0, 100.0]:
            _say(f"threshold mixed wpl={wpl} pct={pct}")
            b.set_threshold(pct)
            b.run()
            ok, lens = b.decisions()
            _check(pairs, sim, L, pct, ok, lens)
            if pct == 0.0:
                assert (lens == UNKNOWN).all()      # settled before any column
            early += int((lens == UNKNOWN).sum())
            # lcs_batch_lengths reports the same lengths
            assert np.array_equal(b.lengths(), lens)
    # pairs far from the threshold stop before their last column
    assert early > len(pairs) * 2


def test_threshold_stops_long_pairs_early(ctx, lcs):
    # unrelated long pairs keep about two thirds of X: a 90% threshold is
    # out of reach long before the last column, and 40% is reached early
    g = inputs.rng(8200)
    pairs = []
    for m in [9000, 30000, 60000]:
        pairs.append((inputs.random_seq(g, m, inputs.DNA).tobytes(),
                      inputs.random_seq(g, m, inputs.DNA).tobytes()))
    sim = _similarity(pairs)
    for pct in (90.0, 40.0):
        _say(f"threshold long unrelated pct={pct}")
        ok, lens = lcs.lcs_threshold_batch(ctx, pairs, pct, "dna")
        assert np.array_equal(ok, sim >= pct)
        assert (lens == UNKNOWN).all()


def test_threshold_boundaries_exact(ctx, lcs, mixed):
    # a threshold equal to the pair's own percentage passes, the next double
    # up fails; targets change between runs of one resident batch
    pairs, sim, L = mixed
    idx = [0, 5, 17, 40, 69, 70, 72, 74, 75]
    for k in idx:
        _say(f"threshold boundary pair {k} m={len(pairs[k][0])} n={len(pairs[k][1])}")
        with lcs.Batch(ctx, [pairs[k]], "dna", threshold=sim[k]) as b:
            b.run()
            ok, lens = b.decisions()
            assert ok[0] and lens[0] in (L[k], UNKNOWN)
            b.set_threshold(float(np.nextafter(sim[k], np.inf)) if sim[k] < 100.0 else 100.0)
            b.run()
            ok2, lens2 = b.decisions()
            assert ok2[0] == (sim[k] >= 100.0) and lens2[0] in (L[k], UNKNOWN)


def test_threshold_graph_and_plain(ctx, lcs, mixed):
    pairs, sim, L = mixed
    sub = pairs[60:]
    s2, L2 = sim[60:], L[60:]
    _say("threshold graph replays")
    with lcs.Batch(ctx, sub, "dna", graph=True, threshold=85.0) as b:
        for pct in (85.0, 70.0, 85.0, 97.0):
            b.set_threshold(pct)
            b.run()
            ok, lens = b.decisions()
            _check(sub, s2, L2, pct, ok, lens)
    _say("threshold plain per-pair launches")
    with lcs.Batch(ctx, sub, "dna", plain=True, threshold=80.0) as b:
        b.run()
        ok, lens = b.decisions()
        _check(sub, s2, L2, 80.0, ok, lens)


def test_threshold_edges(ctx, lcs):
    pairs = [(b"", b""), (b"", b"ACGT"), (b"ACGT", b""), (b"A", b"A"), (b"A", b"C"),
             (b"ACGT" * 40, b"ACGT" * 40), (b"AC" * 100, b"GT" * 100)]
    sim = _similarity(pairs)
    assert list(sim[:3]) == [100.0, 100.0, 0.0]
    for pct in (0.0, 0.5, 50.0, 100.0):
        _say(f"threshold edges pct={pct}")
        ok, lens = lcs.lcs_threshold_batch(ctx, pairs, pct, "dna")
        assert np.array_equal(ok, sim >= pct)
    ok, lens = lcs.lcs_threshold_batch(ctx, [], 50.0, "dna")
    assert ok.size == 0 and lens.size == 0
    for bad in (-1.0, 100.5, float("nan")):
        with pytest.raises(lcs.LcsError) as e:
            lcs.lcs_threshold_batch(ctx, pairs, bad, "dna")
        assert e.value.status == lcs.LCS_ERR_ARG
    with pytest.raises(lcs.LcsError) as e:
        lcs.Batch(ctx, pairs, "dna", traceback=True, threshold=50.0)
    assert e.value.status == lcs.LCS_ERR_ARG
    # a threshold batch must be given its threshold before it runs
    b = lcs.Batch(ctx, pairs, "dna")
    with pytest.raises(lcs.LcsError):
        b.set_threshold(50.0)        # not a threshold batch
    b.close()


def test_similarity_batch_bit_exact(ctx, lcs, mixed):
    pairs, sim, _ = mixed
    _say("similarity batch")
    got = lcs.lcs_similarity_batch(ctx, pairs + [(b"", b"ACG"), (b"ACG", b"")], "dna")
    want = np.concatenate([sim, [100.0, 0.0]])
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


def test_threshold_related_workload_4096(ctx, lcs):
    # the 4096-pair related workload at three thresholds: a sample of pairs
    # against the oracle, every reported length within its bounds and
    # consistent with its answer
    ps = inputs.batch_related()
    pairs = [(p.x, p.y) for p in ps]
    m = np.array([len(p.x) for p in ps])
    n = np.array([len(p.y) for p in ps])
    order = np.argsort(m * n)
    sample = list(order[:40]) + list(order[::400]) + list(order[-3:])
    sp = [(pairs[k][0].tobytes(), pairs[k][1].tobytes()) for k in sample]
    ssim = _similarity(sp)
    with lcs.Batch(ctx, pairs, "dna", graph=True, threshold=90.0) as b:
        for pct in (80.0, 90.0, 95.0):
            _say(f"threshold related 4096 pct={pct}")
            b.set_threshold(pct)
            b.run()
            ok, lens = b.decisions()
            assert np.array_equal(ok[sample], ssim >= pct)
            known = lens != UNKNOWN
            assert (lens[known] <= np.minimum(m, n)[known]).all()
            pk = (100.0 * lens[known].astype(np.float64)) / m[known]
            assert np.array_equal(ok[known], pk >= pct)


@pytest.mark.parametrize("sigma", [20, 150, 256])
def test_threshold_wide_alphabets(ctx, lcs, sigma):
    # protein codes, and alphabets whose stream holds plain codes (above 127
    # symbols at one or two words per lane): short, single-wave and chained
    # pairs, related and unrelated
    g = inputs.rng(8300 + sigma)
    syms = inputs.PROTEIN if sigma == 20 else bytes(range(sigma))
    alpha = "protein" if sigma == 20 else (None if sigma == 256 else syms)
    pairs = []
    for k, m in enumerate([40, 300, 900, 2500, 6000, 9000, 17000]):
        x = inputs.random_seq(g, m, syms)
        if k % 2:
            y, _ = inputs.mutate(g, x, float(g.uniform(0.05, 0.4)), syms)
        else:
            y = inputs.random_seq(g, m, syms)
        pairs.append((x.tobytes(), y.tobytes()))
    sim, L = _similarity(pairs), _lengths(pairs)
    # (at 256 symbols two words per lane need more LDS than a work-group has)
    for wpl in ((1,) if sigma == 256 else (1, 2)):
        with lcs.Batch(ctx, pairs, alpha, threshold=50.0, words_per_lane=wpl) as b:
            for pct in (5.0, 50.0, 80.0, 95.0):
                _say(f"threshold sigma={sigma} wpl={wpl} pct={pct}")
                b.set_threshold(pct)
                b.run()
                ok, lens = b.decisions()
                _check(pairs, sim, L, pct, ok, lens)
