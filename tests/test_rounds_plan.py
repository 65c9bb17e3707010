"""Planner of the traceback in rounds (host only, no device).

Every plan passes the library's self-check, which verifies that each work
item is refilled in exactly one round within the round capacity, that a
chain's items are taken top-down, that every strip is walked once in the
round of the items holding it (group tops below a pair's top strip starting
from the strip above), and the fix-up and seal tickets of every group.
"""
import numpy as np
import pytest

from paper_1306_4627_amd import inputs, lcs


def _plans(m, n, sigma, kibs, **tuning):
    # rounds keep chains unlinked: compare with the fast form packed the same way
    full = lcs.plan_describe(m, n, sigma, traceback=True, **{"link_items": 1, **tuning})
    out = []
    for kib in kibs:
        try:
            d = lcs.plan_describe(m, n, sigma, traceback=True, tb_round_kib=kib, **tuning)
        except lcs.LcsError as e:
            assert e.status == lcs.LCS_ERR_NOMEM
            continue
        assert lcs.plan_selfcheck(m, n, sigma, traceback=True, tb_round_kib=kib, **tuning) == 0
        assert d["history_bytes"] <= kib * 1024 + 8
        assert d["lane_steps"] == full["lane_steps"]       # same packing as the full form
        out.append((kib, d))
    return full, out


def test_long_related_pair_rounds():
    # 262144 rows at one word per lane: 64 items of about 4 MiB of history
    full, out = _plans([262144], [262300], 4, (1024, 4500, 8192, 65536, 300000), words_per_lane=1)
    got = {k: d["tb_rounds"] for k, d in out}
    assert 1024 not in got                      # one item does not fit 1 MiB
    assert got[4500] == 64 and got[8192] == 64  # one item per round
    assert got[65536] == 5                      # 15 items per round
    assert got[300000] == 1
    assert full["history_bytes"] > 256 << 20


def test_related_batch_rounds():
    ps = inputs.batch_related()
    m = [p.x.size for p in ps]
    n = [p.y.size for p in ps]
    full, out = _plans(m, n, 4, (16 << 10, 256 << 10, 1 << 20))
    assert [d["tb_rounds"] for _, d in out] == sorted((d["tb_rounds"] for _, d in out), reverse=True)
    assert all(d["tb_rounds"] >= 2 for _, d in out)
    assert full["history_bytes"] > 4 << 30


@pytest.mark.parametrize("wpl", [1, 2, 4])
def test_mixed_shapes_rounds(wpl):
    g = np.random.default_rng(5)
    m = list(g.integers(0, 30000 * wpl, 60)) + [0, 1, 64, 4096 * wpl, 4096 * wpl + 1]
    n = list(g.integers(0, 20000, 60)) + [5, 0, 64, 100, 3]
    _, out = _plans(m, n, 4, (64, 256, 1024, 4096), words_per_lane=wpl)
    assert out


def test_rounds_refuse_plain_and_linked_items():
    with pytest.raises(lcs.LcsError):
        lcs.plan_describe([9000], [9000], 4, traceback=True, tb_round_kib=4096, plain=True)
    with pytest.raises(lcs.LcsError):
        lcs.plan_describe([9000, 9000], [9000, 9000], 4, traceback=True, tb_round_kib=4096,
                          link_items=8)
