"""CPU-side checks of the C-ABI library: it loads, exports every function the
header declares, validates arguments before touching a device, and packs
pairs correctly (host-only planner).  No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1306_4627_amd import inputs, lcs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lcs.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lcs_[a-z_]+)\s*\(", text)))


def test_header_symbols_are_exported():
    names = _declared_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lcs.lib(), name), f"{name} declared in lcs.h but not exported"


def test_status_strings_and_version():
    assert lcs.status_str(0) == "ok"
    for code in range(-7, 2):
        assert lcs.status_str(code) and lcs.status_str(code) != "unknown status"
    assert lcs.status_str(-99) == "unknown status"
    assert "gfx950" in lcs.version()


def _no_gpu():
    # the kernel driver's device node; no runtime is initialised to look
    return not os.path.exists("/dev/kfd")


@pytest.mark.skipif(not _no_gpu(), reason="checks the no-device path")
def test_create_without_device_fails_cleanly():
    with pytest.raises(lcs.LcsError) as e:
        lcs.Context(0)
    assert e.value.status == lcs.LCS_ERR_DEVICE


def test_autotune_arguments_rejected_before_any_device_call():
    L = lcs.lib()
    best = lcs.lcs_tuning()
    al = lcs.lcs_alphabet(4, ctypes.cast(ctypes.c_char_p(b"ACGT"), ctypes.POINTER(ctypes.c_uint8)))
    assert L.lcs_autotune(None, None, 0, ctypes.byref(al), 0, ctypes.byref(best), None) == lcs.LCS_ERR_ARG


def test_server_arguments_rejected_before_any_device_call():
    L = lcs.lib()
    h = ctypes.c_void_p()
    assert L.lcs_server_create(None, None, ctypes.byref(h)) == lcs.LCS_ERR_ARG
    t = ctypes.c_uint64(0)
    al = lcs.lcs_alphabet(4, ctypes.cast(ctypes.c_char_p(b"ACGT"), ctypes.POINTER(ctypes.c_uint8)))
    assert L.lcs_submit(None, None, 0, None, 0, ctypes.byref(al), 0, ctypes.byref(t)) == lcs.LCS_ERR_ARG
    assert L.lcs_poll(None, 1) == lcs.LCS_ERR_ARG
    assert L.lcs_wait(None, 1, 0) == lcs.LCS_ERR_ARG
    assert L.lcs_cancel(None, 1) == lcs.LCS_ERR_ARG
    assert L.lcs_result(None, 1, ctypes.byref(t), None, 0, None) == lcs.LCS_ERR_ARG
    assert lcs.status_str(lcs.LCS_PENDING).startswith("pending")
    L.lcs_server_destroy(None)


def test_threshold_arguments_and_flags_rejected_before_any_device_call():
    L = lcs.lib()
    al = lcs.lcs_alphabet(4, ctypes.cast(ctypes.c_char_p(b"ACGT"), ctypes.POINTER(ctypes.c_uint8)))
    ok = (ctypes.c_uint8 * 1)()
    n = (ctypes.c_uint64 * 1)()
    pct = (ctypes.c_double * 1)()
    assert L.lcs_threshold_batch(None, None, 0, ctypes.byref(al), 50.0, ok, n) == lcs.LCS_ERR_ARG
    assert L.lcs_similarity_batch(None, None, 0, ctypes.byref(al), pct) == lcs.LCS_ERR_ARG
    assert L.lcs_batch_set_threshold(None, 50.0) == lcs.LCS_ERR_ARG
    assert L.lcs_batch_decisions(None, ok, n) == lcs.LCS_ERR_ARG
    mhz = ctypes.c_double()
    assert L.lcs_batch_clock(None, ctypes.byref(mhz)) == lcs.LCS_ERR_ARG
    # the threshold pass plans like a lengths-only pass; never with a traceback
    m = np.array([100, 9000], dtype=np.uint64)
    P64 = ctypes.POINTER(ctypes.c_uint64)
    s = lcs.lcs_batch_stats()
    t = lcs.lcs_tuning()
    mp = m.ctypes.data_as(P64)
    assert L.lcs_plan_describe(mp, mp, 2, 4, lcs.LCS_THRESHOLD, ctypes.byref(t),
                               ctypes.byref(s)) == lcs.LCS_OK
    assert L.lcs_plan_describe(mp, mp, 2, 4, lcs.LCS_THRESHOLD | lcs.LCS_WANT_TRACEBACK,
                               ctypes.byref(t), ctypes.byref(s)) == lcs.LCS_ERR_ARG
    assert L.lcs_plan_describe(mp, mp, 2, 4, 16, ctypes.byref(t), ctypes.byref(s)) == lcs.LCS_ERR_ARG
    best = lcs.lcs_tuning()
    assert L.lcs_autotune(None, None, 0, ctypes.byref(al), lcs.LCS_THRESHOLD, ctypes.byref(best),
                          None) == lcs.LCS_ERR_ARG
    # schedule records plan like the pass they trace; the autotuner does not take them
    for f in (0, lcs.LCS_WANT_TRACEBACK, lcs.LCS_THRESHOLD):
        assert L.lcs_plan_describe(mp, mp, 2, 4, f | lcs.LCS_FILL_TRACE, ctypes.byref(t),
                                   ctypes.byref(s)) == lcs.LCS_OK
    assert L.lcs_autotune(None, None, 0, ctypes.byref(al), lcs.LCS_FILL_TRACE, ctypes.byref(best),
                          None) == lcs.LCS_ERR_ARG
    cnt = ctypes.c_uint64(5)
    assert L.lcs_batch_fill_trace(None, None, 0, ctypes.byref(cnt)) == lcs.LCS_ERR_ARG
    assert cnt.value == 5


def test_null_arguments_rejected_before_any_device_call():
    L = lcs.lib()
    out = ctypes.c_uint64(7)
    al = lcs.lcs_alphabet(4, ctypes.cast(ctypes.c_char_p(b"ACGT"), ctypes.POINTER(ctypes.c_uint8)))
    assert L.lcs_length(None, None, 0, None, 0, ctypes.byref(al), ctypes.byref(out)) == lcs.LCS_ERR_ARG
    assert out.value == 7   # untouched on error
    assert L.lcs_create(None, 0, 0) == lcs.LCS_ERR_ARG
    assert L.lcs_set_stream(None, None) == lcs.LCS_ERR_ARG
    assert L.lcs_synchronize(None) == lcs.LCS_ERR_ARG
    assert L.lcs_batch_run(None) == lcs.LCS_ERR_ARG
    assert L.lcs_batch_info(None, None) == lcs.LCS_ERR_ARG
    L.lcs_destroy(None)
    L.lcs_batch_destroy(None)


def test_plan_rejects_bad_tuning_and_alphabets():
    m, n = [100, 200], [300, 50]
    with pytest.raises(lcs.LcsError) as e:
        lcs.plan_describe(m, n, 4, words_per_lane=3)
    assert e.value.status == lcs.LCS_ERR_ARG
    with pytest.raises(lcs.LcsError) as e:
        lcs.plan_describe(m, n, 4, traceback=True, ckpt_interval=100)
    assert e.value.status == lcs.LCS_ERR_ARG
    with pytest.raises(lcs.LcsError) as e:
        lcs.plan_describe(m, n, 200, words_per_lane=4)   # plain codes: one or two words per lane
    assert e.value.status == lcs.LCS_ERR_UNSUPPORTED
    with pytest.raises(lcs.LcsError) as e:
        lcs.plan_describe(m, n, 256, words_per_lane=2)   # 257 x 1 KiB of match masks per wave
    assert e.value.status == lcs.LCS_ERR_UNSUPPORTED
    # one wave's LDS is its match masks plus 512 bytes of threshold-pass
    # words: 160 symbols x 1 KiB + 512 B no longer fits 160 KiB
    assert lcs.plan_describe(m, n, 158, words_per_lane=2)["words_per_lane"] == 2
    with pytest.raises(lcs.LcsError) as e:
        lcs.plan_describe(m, n, 159, words_per_lane=2)
    assert e.value.status == lcs.LCS_ERR_UNSUPPORTED
    with pytest.raises(lcs.LcsError) as e:
        lcs.plan_describe(m, n, 20, words_per_lane=8)
    assert e.value.status == lcs.LCS_ERR_UNSUPPORTED
    # every alphabet size up to all 256 bytes is planned (one word per lane
    # at the largest sizes)
    for sigma in (1, 4, 20, 79, 80, 127, 128, 159, 200, 256):
        d = lcs.plan_describe(m, n, sigma, traceback=True)
        assert d["words_per_lane"] >= 1
        assert lcs.plan_selfcheck([1, 64, 700, 5000, 70000], [9, 64, 800, 4000, 100], sigma,
                                  traceback=True) == 0
    with pytest.raises(lcs.LcsError) as e:
        lcs.plan_describe([1 << 40], [5], 4)
    assert e.value.status == lcs.LCS_ERR_TOO_LONG


@pytest.mark.parametrize("wpl", [0, 1, 2, 4, 8])
@pytest.mark.parametrize("tb", [False, True])
def test_packer_edge_lengths(wpl, tb):
    lens = [0, 1, 2, 63, 64, 65, 127, 128, 129, 4095, 4096, 4097, 16384, 16385, 70000]
    m = [a for a in lens for _ in lens]
    n = [b for _ in lens for b in lens]
    assert lcs.plan_selfcheck(m, n, 4, traceback=tb, words_per_lane=wpl) == 0
    d = lcs.plan_describe(m, n, 4, traceback=tb, words_per_lane=wpl)
    assert d["cells"] == sum(a * b for a, b in zip(m, n))
    assert d["pairs"] == len(m)


def test_packer_plain_mode_one_pair_per_item():
    g = np.random.default_rng(0)
    m = g.integers(1, 3000, size=200)
    n = g.integers(1, 3000, size=200)
    assert lcs.plan_selfcheck(m, n, 4, plain=True) == 0
    d = lcs.plan_describe(m, n, 4, plain=True, words_per_lane=1)
    # every pair of at most 64 lanes owns a whole item
    assert d["groups"] >= 200


def test_packer_plain_traceback_tickets_per_pair():
    # plain mode launches one pair's strips of a pass as one ticket range; the
    # packed mode orders the speculative strips longest first across pairs
    g = np.random.default_rng(1)
    m = g.integers(1, 5000, size=120)
    n = g.integers(1, 5000, size=120)
    for wpl in (1, 2):
        for plain in (True, False):
            assert lcs.plan_selfcheck(m, n, 4, traceback=True, plain=plain, words_per_lane=wpl,
                                      strip_rows=512) == 0, (wpl, plain)


def test_packer_short_batch_full_size():
    ps = inputs.batch_short(65536)
    m = [p.x.size for p in ps]
    n = [p.y.size for p in ps]
    for w in (0, 1, 2):
        assert lcs.plan_selfcheck(m, n, 20, words_per_lane=w) == 0
    d = lcs.plan_describe(m, n, 20)
    useful = sum(a * b for a, b in zip(m, n))
    # lane-steps hold 64 cells each; packing keeps most of them busy
    assert useful / (d["lane_steps"] * 64) > 0.7


def test_packer_related_batch_full_size():
    rng = np.random.Generator(np.random.PCG64(inputs.BASE_SEED + 41))
    lx = np.floor(np.exp(rng.uniform(np.log(256), np.log(65536), size=4096))).astype(np.int64)
    ly = (lx * rng.uniform(0.9, 1.1, size=4096)).astype(np.int64)
    for w in (0, 1, 4, 8):
        assert lcs.plan_selfcheck(lx, ly, 4, traceback=True, words_per_lane=w) == 0


def test_packer_long_pair_chains():
    for w in (1, 2, 4, 8):
        assert lcs.plan_selfcheck([262144], [262144 + 77], 4, traceback=True, words_per_lane=w) == 0
        d = lcs.plan_describe([262144], [262144], 4, words_per_lane=w)
        assert d["groups"] == -(-262144 // (64 * 64 * w))


@pytest.mark.parametrize("strip_rows", [0, 1, 64, 100, 2048, 10 ** 6])
def test_traceback_strip_tables(strip_rows):
    # every strip walked once speculatively, every strip below a pair's top
    # one fixed up once, one seal per pair with two or more strips
    m = [1, 63, 64, 65, 128, 129, 4095, 4096, 4097, 10000, 70000, 262144]
    n = [5, 64, 1, 70, 128, 3000, 4096, 100, 4097, 9000, 65000, 262144 + 77]
    for w in (1, 2, 4, 8):
        assert lcs.plan_selfcheck(m, n, 4, traceback=True, words_per_lane=w,
                                  strip_rows=strip_rows) == 0


def _header_struct_fields(name):
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + r"\s*;", text).group(1)
    return [re.findall(r"(\w+)\s*;", line)[0] for line in body.splitlines() if ";" in line]


@pytest.mark.parametrize("name", ["lcs_tuning", "lcs_batch_stats", "lcs_pair"])
def test_binding_structs_mirror_the_header(name):
    # the ctypes mirrors list the header's fields in the header's order
    ours = [f for f, _ in getattr(lcs, name)._fields_]
    assert ours == _header_struct_fields(name)


def test_halves_setting_is_checked():
    L = lcs.lib()
    m = np.array([5000, 9000], dtype=np.uint64)
    P64 = ctypes.POINTER(ctypes.c_uint64)
    mp = m.ctypes.data_as(P64)
    s = lcs.lcs_batch_stats()
    for hv, want in ((0, lcs.LCS_OK), (1, lcs.LCS_OK), (2, lcs.LCS_OK), (3, lcs.LCS_ERR_ARG),
                     (-1, lcs.LCS_ERR_ARG)):
        t = lcs.lcs_tuning()
        t.halves = hv
        assert L.lcs_plan_describe(mp, mp, 2, 4, 0, ctypes.byref(t), ctypes.byref(s)) == want
