"""The early-exit rule of the threshold pass, checked on the CPU against the
oracle's full c table (section I.C).

The fill keeps the rows of a pair in blocks (one block per lane), lanes in
work items of G lanes, and runs lane l of item h with a skew of
h*(G-1+C) + l steps (C steps per chunk).  At the start of chunk c (every
E-th chunk, item h at the chunks c = h mod E) an item adds the zero bits of
its lanes (block k at column j holds
c[top_k][j] - c[bottom_k - 1][j] of them) to the running sum handed up from
the item below at the start of the previous chunk.  The pair's top lane then
knows a sum H and two columns: J, its own, and Jb, the bottom lane's at the
snapshot that entered H.  The rule claims

    H - (Jb - J) <= c[m][J] <= H,

so the pair passes a target T once H - (Jb - J) >= T, and fails once
H + (n - J) < T.  These tests rebuild H exactly as the kernel forms it and
check the claim at every snapshot, and that every early answer is the final
one, over many shapes.
"""
import numpy as np
import pytest

import oracle
from paper_1306_4627_amd import inputs


def _clamp(j, n):
    return min(max(j, 0), n)


def _snapshots(c_tab, R, G, C, E=1):
    """(H, J, Jb) at the chunks where the top item checks, as its top lane
    sees them.  Item h forms its sum only at the chunks c = h (mod E), from
    the sum its feeder formed at chunk c - 1 (which must exist: a KeyError
    here would mean the schedule hands up a sum that was never formed)."""
    m, n = c_tab.shape[0] - 1, c_tab.shape[1] - 1
    lanes = -(-m // R)
    K, l_top = (lanes - 1) // G, (lanes - 1) % G
    step = G - 1 + C
    steps = n + K * step + l_top + 1
    nch = -(-steps // C)

    def zeros(lane, j):
        j = _clamp(j, n)
        lo, hi = lane * R, min(m, lane * R + R)
        return int(c_tab[hi, j]) - int(c_tab[lo, j])

    H = {}
    out = []
    for c in range(nch):
        for h in range(K + 1):
            if (c - h) % E:
                continue
            s = sum(zeros(h * G + l, C * c - (h * step + l))
                    for l in range(G) if h * G + l < lanes)
            # below chunk 0 nothing has been handed up yet
            H[h, c] = s + (H[h - 1, c - 1] if h > 0 and c > 0 else 0)
        if (c - K) % E == 0:
            J = _clamp(C * c - (K * step + l_top), n)
            Jb = _clamp(C * (c - K), n)
            out.append((H[K, c], J, Jb))
    return out


def _pairs(seed, count):
    g = inputs.rng(seed)
    out = []
    for k in range(count):
        m = int(g.integers(1, 160))
        n = int(g.integers(0, 120))
        x = inputs.random_seq(g, m, inputs.DNA)
        if k % 2:
            y, _ = inputs.mutate(g, x, float(g.uniform(0.02, 0.4)), inputs.DNA)
        else:
            y = inputs.random_seq(g, n, inputs.DNA)
        out.append((x.tobytes(), y.tobytes()))
    return out


@pytest.mark.parametrize("R,G,C,E", [(1, 1, 1, 1), (3, 2, 4, 1), (8, 4, 8, 1), (5, 3, 2, 1),
                                     (2, 4, 1, 1), (16, 2, 16, 1), (3, 2, 4, 4), (2, 3, 2, 3),
                                     (4, 2, 2, 4)])
def test_staircase_sum_brackets_the_top_row(R, G, C, E):
    for x, y in _pairs(900 + 7 * R + G + C + E, 40):
        c_tab, _ = oracle.lcs_tables(x, y)
        m = len(x)
        for H, J, Jb in _snapshots(c_tab, R, G, C, E):
            assert 0 <= Jb - J
            assert H - (Jb - J) <= int(c_tab[m, J]) <= H, (len(x), len(y), H, J, Jb)
            if J == Jb == len(y):
                # every lane past the last column: the sum is the length
                assert H == int(c_tab[m, len(y)])


@pytest.mark.parametrize("R,G,C,E", [(4, 2, 4, 1), (8, 4, 8, 1), (2, 3, 2, 1), (2, 3, 2, 4)])
def test_early_answers_are_final_and_happen(R, G, C, E):
    early = 0
    total = 0
    for x, y in _pairs(1900 + R + G + C + E, 40):
        c_tab, _ = oracle.lcs_tables(x, y)
        m, n = len(x), len(y)
        L = int(c_tab[m, n])
        snaps = _snapshots(c_tab, R, G, C, E)
        for T in range(0, min(m, n) + 1):
            for k, (H, J, Jb) in enumerate(snaps):
                yes = H - (Jb - J) >= T
                no = H + (n - J) < T
                assert not (yes and no)
                if yes or no:
                    assert yes == (L >= T), (m, n, T, k)
                    early += k < len(snaps) - 1
                    break
            total += 1
    # a good share of the answers comes before the last chunk
    assert early > total // 4


def test_similarity_and_threshold_pins():
    # closed cases of the percentage and of the yes/no question
    assert oracle.similarity_percent(b"ACGTACGT", b"ACGTACGT") == 100.0
    assert oracle.similarity_percent(b"ACG", b"TTATCTTG") == 100.0      # X inside Y
    assert oracle.similarity_percent(b"AAAA", b"CCGT") == 0.0
    assert oracle.similarity_percent(b"ACGT", b"") == 0.0
    assert oracle.similarity_percent(b"", b"ACGT") == 100.0
    assert oracle.similarity_percent(b"", b"") == 100.0
    # L = 1 of m = 3 (brute force agrees)
    assert oracle.brute_force_length(b"ACG", b"TTA") == 1
    assert oracle.similarity_percent(b"ACG", b"TTA") == 100.0 / 3.0
    # the reported percentage passes its own threshold; the next double up fails
    g = inputs.rng(2300)
    for _ in range(200):
        x = inputs.random_seq(g, int(g.integers(1, 40)), inputs.DNA).tobytes()
        y = inputs.random_seq(g, int(g.integers(0, 40)), inputs.DNA).tobytes()
        p = oracle.similarity_percent(x, y)
        assert oracle.threshold_pass(x, y, p)
        assert not oracle.threshold_pass(x, y, float(np.nextafter(p, np.inf)))
        assert oracle.threshold_pass(x, y, 0.0)
        assert oracle.threshold_pass(x, y, 100.0) == (oracle.brute_force_length(x, y) == len(x)
                                                       if len(x) <= 14 else p == 100.0)
