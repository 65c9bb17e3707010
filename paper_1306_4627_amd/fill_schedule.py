"""Summaries of a fill pass's schedule records (``lcs_batch_fill_trace``).

Host-side arithmetic over the per-item records only: how many wavefronts
were running over the pass, how long the pass ran with fewer than nearly all
of them, how much of the items' time went to building match masks and to
waiting for a feeding item's carries, and how evenly the SIMDs were loaded.
"""
from __future__ import annotations

from typing import Dict

import numpy as np


def simd_key(hw_id: np.ndarray, xcc_id: np.ndarray) -> np.ndarray:
    """A number unique to each SIMD, from the HW_ID and XCC_ID registers:
    die, shader engine, shader array, CU and SIMD fields (not dense)."""
    hw = hw_id.astype(np.int64)
    simd = (hw >> 4) & 3
    cu = (hw >> 8) & 15
    sh = (hw >> 12) & 1
    se = (hw >> 13) & 7
    xcc = xcc_id.astype(np.int64) & 15
    return (((xcc * 8 + se) * 2 + sh) * 16 + cu) * 4 + simd


def concurrency(start: np.ndarray, end: np.ndarray):
    """(times, running): the number of items running from each event time on."""
    t = np.concatenate([start, end]).astype(np.int64)
    d = np.concatenate([np.ones(len(start), np.int64), -np.ones(len(end), np.int64)])
    o = np.lexsort((d, t))          # ends before starts at equal times
    return t[o], np.cumsum(d[o])


def chain_depth(feeder: np.ndarray) -> np.ndarray:
    """Place of each item in its chain (0: fed by no item), from the feeder
    links; a feeder always comes earlier in the queue."""
    d = np.zeros(len(feeder), dtype=np.int64)
    for k, f in enumerate(feeder.tolist()):
        if f >= 0:
            d[k] = d[f] + 1
    return d


def summarize(rec: np.ndarray, near_full: float = 0.9) -> Dict[str, float]:
    """Figures of one pass (records as returned by ``Batch.fill_trace``).

    span_ms            first item taken to last item done
    items, simds       items that ran; SIMDs that ran them
    peak_waves         most items running at once (the resident wave slots used)
    mean_waves         item-time over the span (average running items)
    tail_frac          share of the span after the last instant at which at
                       least ``near_full`` x peak_waves items were running
    setup_frac         share of item-time before the first column step (queue
                       ticket, lane tables, match masks)
    wait_frac          share of the column-step time of items with a feeder
                       spent waiting for its carries
    simd_steps_spread  max over mean of the column steps each SIMD ran
    simd_end_spread    (last - first) SIMD finishing time over the span
    wait_frac_by_depth wait_frac of the items at places 1, 2, ... of their
                       chains (a chain runs at the pace of its slowest item)
    """
    depth_all = chain_depth(rec["feeder"])
    r = rec[rec["ran"] != 0]
    depth = depth_all[rec["ran"] != 0]
    if len(r) == 0:
        return {"items": 0}
    s = r["start_ns"].astype(np.int64)
    f = r["first_step_ns"].astype(np.int64)
    e = r["end_ns"].astype(np.int64)
    w = r["wait_ns"].astype(np.int64)
    span = int(e.max() - s.min())
    t, run = concurrency(s, e)
    peak = int(run.max())
    full = np.nonzero(run >= near_full * peak)[0]
    last_full = int(t[full[-1]]) if len(full) else int(s.min())
    busy = float((e - s).sum())
    chained = r["feeder"] >= 0
    steps_time = (e - f)[chained].sum()
    key = simd_key(r["hw_id"], r["xcc_id"])
    u, inv = np.unique(key, return_inverse=True)
    steps = np.bincount(inv, weights=r["steps"].astype(np.float64))
    simd_end = np.full(len(u), -1, np.int64)
    np.maximum.at(simd_end, inv, e)
    return {
        "span_ms": span / 1e6,
        "items": int(len(r)),
        "simds": int(len(u)),
        "peak_waves": peak,
        "mean_waves": busy / span if span else 0.0,
        "tail_frac": (int(e.max()) - last_full) / span if span else 0.0,
        "setup_frac": float((f - s).sum()) / busy if busy else 0.0,
        "wait_frac": float(w[chained].sum()) / float(steps_time) if steps_time else 0.0,
        "simd_steps_spread": float(steps.max() / steps.mean()),
        "simd_end_spread": float(simd_end.max() - simd_end.min()) / span if span else 0.0,
        "wait_frac_by_depth": [
            round(float(w[depth == d].sum()) / float(max(1, (e - f)[depth == d].sum())), 4)
            for d in range(1, int(depth.max()) + 1)],
    }
