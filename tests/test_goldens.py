"""The stored full-size expected values (CPU only).

* Each golden file's input digest equals the digest of what the seeded
  generators produce now, so the files describe the inputs the GPU tests and
  the benchmark use.
* A sample of the stored values is recomputed with the oracle here, so a
  file cannot drift from the oracle unnoticed.
* The writer of the files calls only the oracle and the input generators.
"""
import ast
import os

import numpy as np
import pytest

import golden_data as gd
import oracle
from paper_1306_4627_amd import inputs


def test_writer_uses_only_the_oracle_and_the_generators():
    src = open(os.path.join(gd.HERE, "make_goldens.py")).read()
    mods = set()
    for node in ast.walk(ast.parse(src)):
        if isinstance(node, ast.Import):
            mods.update(a.name for a in node.names)
        elif isinstance(node, ast.ImportFrom):
            mods.add(node.module or "")
            if node.module == "paper_1306_4627_amd":
                assert [a.name for a in node.names] == ["inputs"]
    assert not any("lcs" in m and m != "oracle" for m in mods), mods


def test_pair_dna_4096_golden():
    p = inputs.pair_dna_4096()
    g = gd.pair("pair_dna_4096")
    assert g.input_sha256 == gd.input_digest([(p.x, p.y)])
    assert (g.m, g.n) == (p.x.size, p.y.size)
    s = oracle.lcs_traceback(p.x, p.y)
    assert g.length == len(s) == oracle.lcs_length(p.x, p.y)
    assert g.string_sha256 == gd.string_digest(s)


@pytest.mark.skipif(not gd.exists("full_pair_long_related.txt"), reason="golden not written")
def test_pair_long_related_golden_inputs():
    p = inputs.pair_long_related()
    g = gd.pair("pair_long_related")
    assert g.input_sha256 == gd.input_digest([(p.x, p.y)])
    assert (g.m, g.n) == (p.x.size, p.y.size)
    # the generator's mutation log bounds the length from below
    assert p.x.size - (p.log.substitutions + p.log.deletions) <= g.length <= min(g.m, g.n)


def test_batch_short_golden():
    ps = inputs.batch_short()
    g = gd.batch_short()
    assert g.input_sha256 == gd.input_digest([(p.x, p.y) for p in ps])
    assert g.lengths.size == len(ps)
    rs = np.random.default_rng(3)
    for k in list(rs.choice(len(ps), 48, replace=False)) + [0, len(ps) - 1]:
        assert g.lengths[k] == oracle.lcs_length(ps[k].x, ps[k].y), k


@pytest.mark.skipif(not gd.exists("full_batch_related.txt"), reason="golden not written")
def test_batch_related_golden():
    ps = inputs.batch_related()
    g = gd.batch_related()
    assert g.input_sha256 == gd.input_digest([(p.x, p.y) for p in ps])
    assert np.array_equal(g.m, [p.x.size for p in ps]) and np.array_equal(g.n, [p.y.size for p in ps])
    for p, L in zip(ps, g.lengths):
        assert p.x.size - (p.log.substitutions + p.log.deletions) <= L <= min(p.x.size, p.y.size)
    # the smallest pairs again with the oracle, strings included
    order = np.argsort([p.cells for p in ps])
    for k in order[:24]:
        s = oracle.lcs_traceback(ps[k].x, ps[k].y)
        assert g.lengths[k] == len(s)
        assert g.sha_prefix[k] == gd.string_digest(s)[:32], k


def test_serve_set_golden():
    reqs = inputs.serve_set()
    digest, g = gd.serve_set()
    assert digest == gd.input_digest([(r.x, r.y) for r in reqs])
    assert len(g) == len(reqs)
    for r, e in zip(reqs, g):
        assert (e.alphabet, e.m, e.n, e.traceback) == (r.alphabet, r.x.size, r.y.size, r.want_traceback)
        assert (e.string_sha256 is not None) == r.want_traceback
    # the two smallest requests with traceback, and the smallest without
    tb = sorted((k for k, r in enumerate(reqs) if r.want_traceback),
                key=lambda k: reqs[k].x.size * reqs[k].y.size)[:2]
    nt = min((k for k, r in enumerate(reqs) if not r.want_traceback),
             key=lambda k: reqs[k].x.size * reqs[k].y.size)
    for k in tb:
        s = oracle.lcs_traceback_ckpt(reqs[k].x, reqs[k].y, 256)
        assert (g[k].length, g[k].string_sha256) == (len(s), gd.string_digest(s))
    assert g[nt].length == oracle.lcs_length(reqs[nt].x, reqs[nt].y)
