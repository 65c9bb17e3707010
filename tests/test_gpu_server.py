"""The request server (continuous batching) against the oracle: every result
exact, the same alone and in a mix of sizes, alphabets and traceback
choices, memory-budgeted admission, cancellation and errors."""
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
ALPHA = {"dna": inputs.DNA, "protein": inputs.PROTEIN, "byte": None}


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


def _mix(seed, count, hi, alphabets=("dna", "protein")):
    g = inputs.rng(seed)
    reqs = []
    for k in range(count):
        al = alphabets[k % len(alphabets)]
        syms = ALPHA[al] if ALPHA[al] is not None else bytes(range(256))
        m = int(np.exp(g.uniform(0, np.log(hi))))
        n = int(np.exp(g.uniform(0, np.log(hi))))
        if k % 7 == 0:
            m = 0
        if k % 11 == 0:
            n = 0
        x = inputs.random_seq(g, m, syms)
        if k % 3 == 0 and m > 0:
            y, _ = inputs.mutate(g, x, float(g.uniform(0.05, 0.3)), syms)
        else:
            y = inputs.random_seq(g, n, syms)
        reqs.append((x, y, al, bool(k % 2)))
    return reqs


def _oracle(reqs):
    def one(r):
        x, y, _, tb = r
        if tb:
            s = oracle.lcs_traceback(x, y)
            return len(s), s
        return oracle.lcs_length(x, y), None
    with ThreadPoolExecutor(THREADS) as ex:
        return list(ex.map(one, reqs))


def _run(srv, reqs):
    tickets = [srv.submit(x, y, ALPHA[al] if al != "byte" else None, traceback=tb)
               for x, y, al, tb in reqs]
    out = []
    for t in tickets:
        assert srv.wait(t, 60_000_000) == 0
        L, s, lat = srv.result(t)
        assert lat > 0
        out.append((L, s))
    return out


def test_server_mix_exact_and_same_alone(ctx, lcs):
    reqs = _mix(7100, 120, 4000, alphabets=("dna", "protein", "byte"))
    want = _oracle(reqs)
    _say(f"server mix {len(reqs)} requests")
    with lcs.Server(ctx, mem_budget_bytes=512 << 20) as srv:
        got = _run(srv, reqs)
        st = srv.stats()
    assert got == want
    assert st["completed"] == len(reqs) and st["failed"] == 0 and st["queued"] == 0
    assert st["batches"] >= 2
    # each of a spread of requests alone on a fresh server: the same answer
    _say("server requests alone")
    with lcs.Server(ctx, mem_budget_bytes=64 << 20, streams=1) as srv:
        for k in range(0, len(reqs), 9):
            assert _run(srv, [reqs[k]]) == [want[k]], k


def test_server_admission_under_a_small_arena(ctx, lcs):
    # every request fits the arena alone, the whole set does not: the
    # dispatcher splits batches and waits for memory to come back
    g = inputs.rng(7200)
    reqs = []
    for k in range(24):
        x = inputs.random_seq(g, 6000 + 97 * k, inputs.DNA)
        y, _ = inputs.mutate(g, x, 0.15, inputs.DNA)
        reqs.append((x, y, "dna", k % 2 == 0))
    want = _oracle(reqs)
    _say("server small arena")
    with lcs.Server(ctx, mem_budget_bytes=1 << 20, streams=3) as srv:
        got = _run(srv, reqs)
        st = srv.stats()
    assert got == want
    assert st["arena_peak_bytes"] <= st["arena_bytes"] == 1 << 20
    assert st["batches"] >= 6


def test_server_request_larger_than_the_arena_fails_alone(ctx, lcs):
    g = inputs.rng(7300)
    small = (inputs.random_seq(g, 500, inputs.DNA), inputs.random_seq(g, 400, inputs.DNA))
    big = (inputs.random_seq(g, 300000, inputs.DNA), inputs.random_seq(g, 300000, inputs.DNA))
    _say("server oversized request")
    with lcs.Server(ctx, mem_budget_bytes=1 << 20) as srv:
        tb = srv.submit(*big, "dna", traceback=True)
        ts = srv.submit(*small, "dna", traceback=True)
        assert srv.wait(tb, 60_000_000) == lcs.LCS_ERR_NOMEM
        assert srv.wait(ts, 60_000_000) == 0
        with pytest.raises(lcs.LcsError) as e:
            srv.result(tb)
        assert e.value.status == lcs.LCS_ERR_NOMEM
        L, s, _ = srv.result(ts)
        assert s == oracle.lcs_traceback(*small) and L == len(s)


def test_server_errors_and_cancel(ctx, lcs):
    _say("server errors")
    with lcs.Server(ctx, mem_budget_bytes=16 << 20, streams=1) as srv:
        with pytest.raises(lcs.LcsError) as e:
            srv.submit(b"ACGX", b"ACG", "dna")
        assert e.value.status == lcs.LCS_ERR_SYMBOL
        g = inputs.rng(7400)
        x = inputs.random_seq(g, 20000, inputs.DNA)
        t1 = srv.submit(x, x, "dna", traceback=True)
        t2 = srv.submit(b"ACGT", b"AGT", "dna")
        c = srv.cancel(t2)
        assert c in (lcs.LCS_OK, lcs.LCS_ERR_ARG)   # it may already be running
        if c == lcs.LCS_OK:
            assert srv.poll(t2) == lcs.LCS_ERR_ARG
        else:
            assert srv.wait(t2, 60_000_000) == 0 and srv.result(t2)[0] == 3
        assert srv.wait(t1, 60_000_000) == 0
        L, s, _ = srv.result(t1)
        assert s == x.tobytes() and L == x.size
        assert srv.poll(t1) == lcs.LCS_ERR_ARG      # collected tickets are gone


def test_server_reuses_the_autotuners_tuning(ctx, lcs):
    # a tuning found for graph replay is cached under the batch's shape
    # without the graph flag, so the server's eager batch of the same shape
    # (one request alone) launches with it
    g = inputs.rng(7500)
    x = inputs.random_seq(g, 30000, inputs.DNA)
    y, _ = inputs.mutate(g, x, 0.1, inputs.DNA)
    _say("server reuses a cached tuning")
    lcs.autotune(ctx, [(x, y)], "dna", traceback=True, graph=True)
    with lcs.Server(ctx, mem_budget_bytes=256 << 20, streams=1) as srv:
        t = srv.submit(x, y, "dna", traceback=True)
        assert srv.wait(t, 60_000_000) == 0
        L, s, _ = srv.result(t)
        st = srv.stats()
    assert st["batches"] == 1 and st["tuned_batches"] == 1
    assert s == oracle.lcs_traceback(x, y) and L == len(s)


def _check_golden(k, e, L, s):
    assert L == e.length, f"request {k}: length {L} != {e.length}"
    if e.traceback:
        assert s is not None and gd.string_digest(s) == e.string_sha256, f"request {k}: string differs"
    else:
        assert s is None


def test_server_serving_scale_requests_in_a_stream(ctx, lcs):
    # requests of 10^4..10^5 symbols over DNA, protein and all 256 bytes, half
    # with tracebacks, a third related (walks that stay near the diagonal) and
    # the rest unrelated (walks that fall back to the sequential seal); they
    # arrive 3 ms apart, so later ones are admitted while earlier ones run.
    # Every result against the oracle's (stored), in the stream and alone.
    import time
    reqs = inputs.serve_set()
    digest, want = gd.serve_set()
    assert digest == gd.input_digest([(r.x, r.y) for r in reqs]), "input generator changed"
    _say(f"server serving-scale stream, {len(reqs)} requests")
    with lcs.Server(ctx, mem_budget_bytes=4 << 30) as srv:
        t0 = time.perf_counter()
        tickets = []
        for k, r in enumerate(reqs):
            while time.perf_counter() - t0 < 0.003 * k:
                pass
            tickets.append(srv.submit(r.x, r.y, ALPHA[r.alphabet], traceback=r.want_traceback))
        for k, t in enumerate(tickets):
            assert srv.wait(t, 120_000_000) == 0, k
            L, s, _ = srv.result(t)
            _check_golden(k, want[k], L, s)
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["batches"] >= 2
    assert st["max_inflight"] >= 2, st      # their work overlapped on the device
    _say("server serving-scale requests alone")
    with lcs.Server(ctx, mem_budget_bytes=4 << 30, streams=1) as srv:
        for k, r in enumerate(reqs):
            t = srv.submit(r.x, r.y, ALPHA[r.alphabet], traceback=r.want_traceback)
            assert srv.wait(t, 120_000_000) == 0, k
            L, s, _ = srv.result(t)
            _check_golden(k, want[k], L, s)
