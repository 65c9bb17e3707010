"""Pins for the CPU oracle, each against something other than the oracle
itself: brute-force enumeration (paper section I), the exponential recursion
(section I.B), hand-worked examples (sections I.C / I.D), closed forms and
invariants that the mathematics fixes, and the generator's mutation log.

All CPU-only.
"""
import functools
import os

import numpy as np
import pytest

import oracle
from paper_1306_4627_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.txt")


def _golden_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            x, y, L, s = line.rstrip("\n").split("\t")
            rows.append((x.encode(), y.encode(), int(L), b"" if s == "-" else s.encode()))
    return rows


def _rand_bytes(g, n, alphabet):
    a = np.frombuffer(alphabet, dtype=np.uint8)
    return bytes(a[g.integers(0, a.size, size=n)])


def canonical_by_definition(x: bytes, y: bytes) -> bytes:
    """The canonical walk written from its definition on prefixes, using
    brute-force LCS lengths (no table): at (i, j) a match emits x_i and goes
    diagonally; otherwise the walk goes up when LCS(X_{i-1}, Y_j) >=
    LCS(X_i, Y_{j-1}) and left otherwise (sections I.C and I.D)."""
    @functools.lru_cache(maxsize=None)
    def L(i, j):
        return oracle.brute_force_length(x[:i], y[:j])

    out = []
    i, j = len(x), len(y)
    while i > 0 and j > 0:
        if x[i - 1] == y[j - 1]:
            out.append(x[i - 1]); i -= 1; j -= 1
        elif L(i - 1, j) >= L(i, j - 1):
            i -= 1
        else:
            j -= 1
    return bytes(reversed(out))


# --------------------------------------------------------------------------
# worked examples
# --------------------------------------------------------------------------

@pytest.mark.parametrize("x,y,L,s", _golden_rows())
def test_worked_examples(x, y, L, s):
    assert oracle.lcs_length(x, y) == L
    assert oracle.lcs_traceback(x, y) == s
    assert oracle.lcs_traceback_ckpt(x, y, 1) == s
    assert oracle.lcs_traceback_ckpt(x, y, 2) == s


@pytest.mark.parametrize("x,y,L,s", _golden_rows())
def test_worked_examples_agree_with_definition(x, y, L, s):
    # the hand-worked answers themselves, re-derived without any table
    assert oracle.brute_force_length(x, y) == L
    assert canonical_by_definition(x, y) == s


def test_swapping_arguments_changes_the_string_not_the_length():
    assert oracle.lcs_traceback(b"AB", b"BA") == b"A"
    assert oracle.lcs_traceback(b"BA", b"AB") == b"B"


# --------------------------------------------------------------------------
# brute force and recursion on tiny inputs
# --------------------------------------------------------------------------

@pytest.mark.parametrize("alphabet", [b"A", b"AB", b"ACGT", b"ACDEFGHIKLMNPQRSTVWY"])
def test_length_matches_brute_force(alphabet):
    g = np.random.default_rng(1)
    for _ in range(60):
        m = int(g.integers(0, 15))
        n = int(g.integers(0, 15))
        x = _rand_bytes(g, m, alphabet)
        y = _rand_bytes(g, n, alphabet)
        assert oracle.lcs_length(x, y) == oracle.brute_force_length(x, y), (x, y)


def test_length_matches_brute_force_at_14():
    g = np.random.default_rng(2)
    for _ in range(6):
        x = _rand_bytes(g, 14, b"ACGT")
        y = _rand_bytes(g, 14, b"ACGT")
        assert oracle.lcs_length(x, y) == oracle.brute_force_length(x, y)


def test_length_matches_recursion():
    g = np.random.default_rng(3)
    for _ in range(40):
        x = _rand_bytes(g, int(g.integers(0, 9)), b"ACG")
        y = _rand_bytes(g, int(g.integers(0, 9)), b"ACG")
        assert oracle.lcs_length(x, y) == oracle.recursive_length(x, y)


def test_traceback_is_a_longest_common_subsequence():
    g = np.random.default_rng(4)
    for _ in range(80):
        x = _rand_bytes(g, int(g.integers(0, 12)), b"ACGT")
        y = _rand_bytes(g, int(g.integers(0, 12)), b"ACGT")
        s = oracle.lcs_traceback(x, y)
        assert s in oracle.brute_force_all_lcs(x, y) or (s == b"" and oracle.brute_force_length(x, y) == 0)


def test_traceback_matches_definition():
    g = np.random.default_rng(5)
    for _ in range(60):
        x = _rand_bytes(g, int(g.integers(0, 10)), b"AB")
        y = _rand_bytes(g, int(g.integers(0, 10)), b"AB")
        assert oracle.lcs_traceback(x, y) == canonical_by_definition(x, y), (x, y)
    for _ in range(40):
        x = _rand_bytes(g, int(g.integers(0, 10)), b"ACGT")
        y = _rand_bytes(g, int(g.integers(0, 10)), b"ACGT")
        assert oracle.lcs_traceback(x, y) == canonical_by_definition(x, y), (x, y)


def test_table_entries_match_brute_force():
    # every c[i][j] is the LCS length of the prefixes X_i, Y_j
    g = np.random.default_rng(6)
    x = _rand_bytes(g, 9, b"ACGT")
    y = _rand_bytes(g, 8, b"ACGT")
    c, b = oracle.lcs_tables(x, y)
    for i in range(len(x) + 1):
        for j in range(len(y) + 1):
            assert c[i, j] == oracle.brute_force_length(x[:i], y[:j])
    # the arrows follow the rule of section I.C
    for i in range(1, len(x) + 1):
        for j in range(1, len(y) + 1):
            if x[i - 1] == y[j - 1]:
                assert b[i, j] == oracle.DIAG
            elif c[i - 1, j] >= c[i, j - 1]:
                assert b[i, j] == oracle.UP
            else:
                assert b[i, j] == oracle.LEFT


# --------------------------------------------------------------------------
# closed forms and invariants
# --------------------------------------------------------------------------

def test_closed_forms():
    g = np.random.default_rng(7)
    x = _rand_bytes(g, 300, b"ACGT")
    assert oracle.lcs_length(x, x) == 300
    assert oracle.lcs_traceback(x, x) == x
    assert oracle.lcs_length(x, b"") == 0
    assert oracle.lcs_length(b"", x) == 0
    assert oracle.lcs_traceback(x, b"") == b""
    assert oracle.lcs_length(_rand_bytes(g, 200, b"AC"), _rand_bytes(g, 200, b"GT")) == 0
    for p, q in [(0, 5), (5, 0), (7, 3), (3, 7), (40, 40)]:
        assert oracle.lcs_length(b"a" * p, b"a" * q) == min(p, q)
    for p, q, r, s in [(3, 5, 2, 4), (6, 1, 1, 6), (0, 4, 4, 0), (5, 5, 5, 5), (2, 9, 3, 1)]:
        X = b"a" * p + b"b" * q
        Y = b"b" * r + b"a" * s
        assert oracle.lcs_length(X, Y) == max(min(p, s), min(q, r))


def test_subsequence_closed_form():
    g = np.random.default_rng(8)
    y = _rand_bytes(g, 500, b"ACGT")
    keep = np.sort(g.choice(500, size=180, replace=False))
    x = bytes(y[k] for k in keep)
    assert oracle.lcs_length(x, y) == len(x)
    assert oracle.lcs_traceback(x, y) == x


def test_invariants_random():
    g = np.random.default_rng(9)
    for _ in range(30):
        m, n = int(g.integers(0, 120)), int(g.integers(0, 120))
        al = [b"AB", b"ACGT", bytes(range(256))][int(g.integers(0, 3))]
        x, y = _rand_bytes(g, m, al), _rand_bytes(g, n, al)
        L = oracle.lcs_length(x, y)
        assert 0 <= L <= min(m, n)
        assert oracle.lcs_length(y, x) == L                       # symmetry
        assert oracle.lcs_length(x[::-1], y[::-1]) == L           # reversal
        s = oracle.lcs_traceback(x, y)
        assert len(s) == L
        assert oracle.is_subsequence(s, x) and oracle.is_subsequence(s, y)
        # appending one symbol changes the length by 0 or 1 (section I.A)
        for extra in (b"A", b"B"):
            d = oracle.lcs_length(x + extra, y) - L
            assert d in (0, 1)


def test_middle_column_split():
    # The reading the lengths-only split rests on (section I.C's table cut at
    # a column h): every path from (0, 0) to (m, n) crosses column h, so
    # L(X, Y) = max over k of L(X[:k], Y[:h]) + L(X[k:], Y[h:]), and the
    # second term is the length of the reversed suffixes.  Checked on the
    # oracle for every h of small pairs, with brute force at the smallest.
    g = np.random.default_rng(12)
    for trial in range(40):
        m, n = int(g.integers(0, 40)), int(g.integers(0, 40))
        al = [b"AB", b"ACGT", b"ACDEFGHIKLMNPQRSTVWY"][trial % 3]
        x, y = _rand_bytes(g, m, al), _rand_bytes(g, n, al)
        L = oracle.lcs_length(x, y)
        for h in range(n + 1):
            best = max(oracle.lcs_length(x[:k], y[:h]) + oracle.lcs_length(x[k:][::-1], y[h:][::-1])
                       for k in range(m + 1))
            assert best == L, (x, y, h)
    x, y = b"ACGTTGCA", b"TTGACCA"
    assert max(oracle.brute_force_length(x[:k], y[:3]) + oracle.brute_force_length(x[k:], y[3:])
               for k in range(len(x) + 1)) == oracle.brute_force_length(x, y)


def test_chvatal_sankoff_range_dna():
    # statistical sanity only: L/n of random DNA pairs sits near 0.654
    p = inputs.pair_dna_4096(2048, 2048)
    L = oracle.lcs_length(p.x, p.y)
    assert 0.62 * 2048 < L < 0.68 * 2048


def test_related_pair_lower_bound():
    # every unmutated symbol of X survives in Y in order, so
    # L >= m - (#substitutions + #deletions)
    g = inputs.rng(1000)
    for rate in (0.05, 0.1, 0.3):
        x = inputs.random_seq(g, 1500, inputs.DNA)
        y, log = inputs.mutate(g, x, rate, inputs.DNA)
        L = oracle.lcs_length(x, y)
        assert L >= x.size - (log.substitutions + log.deletions)
        assert L <= min(x.size, y.size)


# --------------------------------------------------------------------------
# the checkpointed-row oracle against the literal one
# --------------------------------------------------------------------------

@pytest.mark.parametrize("R", [1, 2, 3, 7, 64, 1000])
def test_ckpt_matches_literal_small(R):
    g = np.random.default_rng(10 + R)
    for _ in range(25):
        m, n = int(g.integers(0, 90)), int(g.integers(0, 90))
        al = [b"AB", b"ACGT", b"ACDEFGHIKLMNPQRSTVWY"][int(g.integers(0, 3))]
        x, y = _rand_bytes(g, m, al), _rand_bytes(g, n, al)
        assert oracle.lcs_traceback_ckpt(x, y, R) == oracle.lcs_traceback(x, y)


@pytest.mark.parametrize("m,n,R", [(1024, 1000, 64), (777, 1500, 100), (2048, 2048, 512)])
def test_ckpt_matches_literal_medium(m, n, R):
    g = inputs.rng(2000 + m)
    x = inputs.random_seq(g, m, inputs.DNA)
    y, _ = inputs.mutate(g, x[:n] if n <= m else x, 0.2, inputs.DNA)
    assert oracle.lcs_traceback_ckpt(x, y, R) == oracle.lcs_traceback(x, y)
    assert len(oracle.lcs_traceback(x, y)) == oracle.lcs_length(x, y)


@pytest.mark.slow
def test_ckpt_matches_literal_4096():
    p = inputs.pair_dna_4096()
    assert oracle.lcs_traceback_ckpt(p.x, p.y, 512) == oracle.lcs_traceback(p.x, p.y)


def test_ckpt_rejects_bad_block():
    with pytest.raises(ValueError):
        oracle.lcs_traceback_ckpt(b"AB", b"BA", 0)


# --------------------------------------------------------------------------
# the pins are sharp: a planted mistake in a copy of the oracle's rule fails
# --------------------------------------------------------------------------

def _mutant_traceback(x: bytes, y: bytes, prefer_left: bool) -> bytes:
    c, _ = oracle.lcs_tables(x, y)
    out, i, j = [], len(x), len(y)
    while i > 0 and j > 0:
        if x[i - 1] == y[j - 1]:
            out.append(x[i - 1]); i -= 1; j -= 1
        elif (c[i - 1, j] > c[i, j - 1]) if prefer_left else (c[i - 1, j] >= c[i, j - 1]):
            i -= 1
        else:
            j -= 1
    return bytes(reversed(out))


def test_planted_tie_break_mistake_is_caught():
    rows = _golden_rows()
    good = all(_mutant_traceback(x, y, False) == s for x, y, _, s in rows)
    bad = all(_mutant_traceback(x, y, True) == s for x, y, _, s in rows)
    assert good and not bad


# --------------------------------------------------------------------------
# generator sanity (not the method)
# --------------------------------------------------------------------------

def test_generators_are_seeded_and_shaped():
    a = inputs.pair_dna_4096()
    b = inputs.pair_dna_4096()
    assert a.x.size == 4096 and a.y.size == 4096
    assert np.array_equal(a.x, b.x) and np.array_equal(a.y, b.y)
    assert set(np.unique(a.x).tobytes()) <= set(inputs.DNA)
    bs = inputs.batch_short(200)
    assert all(64 <= p.x.size <= 1024 and 64 <= p.y.size <= 1024 for p in bs)
    assert all(set(np.unique(p.x).tobytes()) <= set(inputs.PROTEIN) for p in bs)
    br = inputs.batch_related(64)
    assert all(256 <= p.x.size <= 65536 for p in br)
    for p in br:
        lg = p.log
        assert p.y.size == p.x.size + lg.insertions - lg.deletions


def test_mutation_rates():
    g = inputs.rng(3000)
    x = inputs.random_seq(g, 200000, inputs.DNA)
    y, lg = inputs.mutate(g, x, 0.1, inputs.DNA)
    tot = lg.substitutions + lg.insertions + lg.deletions
    assert abs(tot / x.size - 0.1) < 0.005
    for k in (lg.substitutions, lg.insertions, lg.deletions):
        assert abs(k / tot - 1 / 3) < 0.02
