"""Host-side summary of fill schedule records (paper_1306_4627_amd.fill_schedule)
on hand-built records whose figures are worked out by hand."""
import numpy as np
import pytest

from paper_1306_4627_amd import fill_schedule
from paper_1306_4627_amd.lcs import FILL_ITEM


def _rec(rows):
    r = np.zeros(len(rows), dtype=FILL_ITEM)
    for k, (s, f, e, w, steps, feeder, hw, ran) in enumerate(rows):
        r[k] = (s, f, e, w, steps, feeder, 0, ran, hw, 0)
    return r


A = 0 << 4           # SIMD 0 of CU 0
B = (1 << 4) | (3 << 8)   # SIMD 1 of CU 3


def test_summary_figures_by_hand():
    r = _rec([
        (0, 100, 1000, 0, 10, -1, A, 1),
        (0, 200, 800, 100, 8, 0, B, 1),
        (800, 850, 1200, 0, 4, -1, B, 1),
        (1000, 1000, 1100, 50, 1, 2, A, 1),
        (5, 5, 99999, 7, 1000, -1, B, 0),      # never ran: ignored
    ])
    s = fill_schedule.summarize(r)
    assert s["items"] == 4 and s["simds"] == 2 and s["peak_waves"] == 2
    assert s["span_ms"] == pytest.approx(1200 / 1e6)
    assert s["mean_waves"] == pytest.approx(2300 / 1200)
    # two items run until t = 1000 (item 0 ends as item 3 starts), then one
    assert s["tail_frac"] == pytest.approx(200 / 1200)
    assert s["setup_frac"] == pytest.approx(350 / 2300)
    assert s["wait_frac"] == pytest.approx(150 / 700)
    assert s["simd_steps_spread"] == pytest.approx(12 / 11.5)
    assert s["simd_end_spread"] == pytest.approx(100 / 1200)


def test_concurrency_counts_ends_before_starts():
    t, run = fill_schedule.concurrency(np.array([0, 10]), np.array([10, 20]))
    assert list(t) == [0, 10, 10, 20] and list(run) == [1, 0, 1, 0]


def test_simd_key_separates_every_field():
    hw = np.array([0, 1 << 4, 1 << 8, 1 << 12, 1 << 13, 0, 15], dtype=np.uint32)
    xcc = np.array([0, 0, 0, 0, 0, 1, 0], dtype=np.uint32)
    k = fill_schedule.simd_key(hw, xcc)
    # wave slot bits (0-3) do not name a SIMD
    assert k[6] == k[0]
    assert len(set(k[:6].tolist())) == 6


def test_chain_depth_and_waits_by_depth():
    # chains 0 -> 1 -> 3 and 2 -> 4; item 5 alone
    r = _rec([
        (0, 0, 100, 0, 1, -1, A, 1),
        (0, 0, 100, 10, 1, 0, A, 1),
        (0, 0, 100, 0, 1, -1, B, 1),
        (0, 0, 100, 30, 1, 1, B, 1),
        (0, 0, 50, 5, 1, 2, A, 1),
        (0, 0, 100, 0, 1, -1, B, 1),
    ])
    assert list(fill_schedule.chain_depth(r["feeder"])) == [0, 1, 0, 2, 1, 0]
    s = fill_schedule.summarize(r)
    assert s["wait_frac_by_depth"] == [pytest.approx(15 / 150), pytest.approx(30 / 100)]
    assert s["wait_frac"] == pytest.approx(45 / 250)


def test_empty_and_unrun():
    assert fill_schedule.summarize(_rec([]))["items"] == 0
    assert fill_schedule.summarize(_rec([(0, 0, 5, 0, 1, -1, A, 0)]))["items"] == 0
