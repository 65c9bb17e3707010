"""Fill schedule records (LCS_FILL_TRACE) on the GPU: a traced batch computes
exactly what the untraced one does (lengths against the oracle, strings
against the untraced batch), every work item is recorded once per pass with
consistent times, feeders and SIMD, also on graph replays, the threshold
pass and the plain per-pair launches."""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_1306_4627_amd import fill_schedule, inputs

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


def _pairs(seed):
    # many short pairs, single-wave pairs and chained pairs (up to 5 items
    # at two words per lane), related and unrelated
    g = inputs.rng(seed)
    out = []
    sizes = [int(np.exp(g.uniform(np.log(16), np.log(4000)))) for _ in range(300)]
    sizes += [8192, 8193, 16000, 30000, 41000]
    for k, m in enumerate(sizes):
        x = inputs.random_seq(g, m, inputs.DNA)
        if k % 3 == 2:
            y = inputs.random_seq(g, int(m * g.uniform(0.6, 1.4)), inputs.DNA)
        else:
            y, _ = inputs.mutate(g, x, float(g.uniform(0.02, 0.3)), inputs.DNA)
        out.append((x.tobytes(), y.tobytes()))
    return out


@pytest.fixture(scope="module")
def mixed():
    p = _pairs(9100)
    with ThreadPoolExecutor(THREADS) as ex:
        L = np.array(list(ex.map(lambda q: oracle.lcs_length(q[0], q[1]), p)), dtype=np.uint64)
    return p, L


def _check_records(rec, info):
    n = len(rec)
    assert n == info["groups"]
    assert (rec["ran"] == 1).all()
    s, f, e, w = (rec[k].astype(np.int64) for k in ("start_ns", "first_step_ns", "end_ns", "wait_ns"))
    assert s.min() == 0
    assert (s <= f).all() and (f <= e).all()
    assert (w <= e - f).all()
    # steps are whole chunks and cover the plan's lane-steps
    assert (rec["steps"] % 64 == 0).all()
    assert int(rec["steps"].astype(np.int64).sum()) * 64 == info["lane_steps"]
    # a chain: the feeder comes earlier in the queue, hands carries on, and
    # starts its column steps before its consumer ends; unchained items never wait
    fd = rec["feeder"]
    ch = np.nonzero(fd >= 0)[0]
    assert (fd[ch] < ch).all()
    assert (rec["feeds"][fd[ch]] == 1).all()
    assert (rec["steps"][fd[ch]] == rec["steps"][ch]).all()
    assert (f[fd[ch]] <= e[ch]).all()
    assert (w[fd < 0] == 0).all()
    assert int((rec["feeds"] == 1).sum()) == len(ch)
    # the SIMD fields decode to one of the chip's 1024 SIMDs (8 dies x 32 CUs x 4)
    assert ((rec["xcc_id"] & 15) < 8).all()
    k = fill_schedule.simd_key(rec["hw_id"], rec["xcc_id"])
    assert len(np.unique(k)) <= 1024
    sm = fill_schedule.summarize(rec)
    assert sm["items"] == n and 1 <= sm["peak_waves"] <= 256 * 16
    for key in ("tail_frac", "setup_frac", "wait_frac", "simd_end_spread"):
        assert 0.0 <= sm[key] <= 1.0, (key, sm[key])
    return sm


@pytest.mark.parametrize("wpl", [1, 2])
def test_traced_batch_matches_untraced_and_oracle(ctx, lcs, mixed, wpl):
    pairs, L = mixed
    _say(f"fill trace: traceback batch wpl={wpl}, untraced")
    with lcs.Batch(ctx, pairs, "dna", traceback=True, words_per_lane=wpl) as b0:
        b0.run()
        s0 = b0.tracebacks()
        assert np.array_equal(b0.lengths(), L)
    _say(f"fill trace: traceback batch wpl={wpl}, traced")
    with lcs.Batch(ctx, pairs, "dna", traceback=True, words_per_lane=wpl, fill_trace=True) as b:
        b.run()
        assert np.array_equal(b.lengths(), L)
        assert b.tracebacks() == s0
        sm = _check_records(b.fill_trace(), b.info())
        _say(f"fill trace summary wpl={wpl}: {sm}")


def test_trace_on_graph_replays_and_lengths_only(ctx, lcs, mixed):
    pairs, L = mixed
    with lcs.Batch(ctx, pairs, "dna", graph=True, fill_trace=True) as b:
        for k in range(3):
            _say(f"fill trace: graph replay {k}")
            b.run()
            assert np.array_equal(b.lengths(), L)
            _check_records(b.fill_trace(), b.info())
        _say("fill trace: eager pass of the graph batch")
        b.time(eager=True)
        assert np.array_equal(b.lengths(), L)
        _check_records(b.fill_trace(), b.info())


def test_trace_threshold_and_plain(ctx, lcs, mixed):
    pairs, L = mixed
    m = np.array([len(x) for x, _ in pairs], dtype=np.float64)
    sim = np.where(m > 0, 100.0 * L.astype(np.float64) / np.maximum(m, 1), 100.0)
    _say("fill trace: threshold pass")
    with lcs.Batch(ctx, pairs, "dna", threshold=70.0, fill_trace=True) as b:
        b.run()
        ok, _ = b.decisions()
        assert np.array_equal(ok, sim >= 70.0)
        rec = b.fill_trace()
        assert len(rec) == b.info()["groups"]
        # items stopped early by an answer still record their times
        assert (rec["ran"] == 1).all()
        assert (rec["start_ns"] <= rec["end_ns"]).all()
    sub = pairs[-40:]
    _say("fill trace: plain per-pair launches")
    with lcs.Batch(ctx, sub, "dna", plain=True, fill_trace=True) as b:
        b.run()
        assert np.array_equal(b.lengths(), L[-40:])
        rec = b.fill_trace()
        assert (rec["ran"] == 1).all() and len(rec) == b.info()["groups"]


def test_trace_requires_flag_and_a_run(ctx, lcs):
    pairs = [(b"ACGT" * 10, b"AGT" * 10)]
    with lcs.Batch(ctx, pairs, "dna") as b:
        b.run()
        with pytest.raises(lcs.LcsError) as e:
            b.fill_trace()
        assert e.value.status == lcs.LCS_ERR_ARG
    with lcs.Batch(ctx, pairs, "dna", fill_trace=True) as b:
        with pytest.raises(lcs.LcsError):
            b.fill_trace()         # before the first run
        b.run()
        assert len(b.fill_trace()) == 1
