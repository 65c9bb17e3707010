"""The host baseline of the paper's row-striped OpenMP method (section II):
the same table and the same canonical walk as the oracle, for every thread
count and chunk width, including more threads than rows."""
import numpy as np
import pytest

import oracle
from paper_1306_4627_amd import inputs
from paper_1306_4627_amd.striped import striped_lcs


@pytest.mark.parametrize("threads", [1, 2, 3, 4, 8])
def test_striped_matches_oracle(threads):
    g = inputs.rng(8100 + threads)
    cases = [(0, 0), (0, 5), (5, 0), (1, 1), (3, 700), (700, 3), (200, 30), (1000, 150), (2000, 200)]
    for m, n in cases:
        for al in (inputs.DNA, b"AB", inputs.PROTEIN):
            x = inputs.random_seq(g, m, al)
            y = inputs.random_seq(g, n, al)
            for chunk in (1, 7, 64):
                L, s, tf, tt = striped_lcs(x, y, threads, chunk)
                assert s == oracle.lcs_traceback(x, y), (m, n, chunk)
                assert L == len(s) and 0 <= tf <= tt


def test_striped_related_pair_and_length_only():
    g = inputs.rng(8200)
    x = inputs.random_seq(g, 5000, inputs.DNA)
    y, _ = inputs.mutate(g, x, 0.2, inputs.DNA)
    L, s, _, _ = striped_lcs(x, y, 4, 64)
    assert s == oracle.lcs_traceback(x, y)
    L2, s2, _, _ = striped_lcs(x, y, 3, 50, traceback=False)
    assert L2 == L and s2 is None
