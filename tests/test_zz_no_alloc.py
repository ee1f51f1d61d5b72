"""The entry point for callers that cannot allocate (fastlec_es_check_noalloc) against the
plain check on the same kernel (fastlec_es_check, interpreter) and against the oracle.

Calls run back to back on one device, each larger one followed by a smaller one, so a call
that read what the previous call left in the shared static array would show up here.
"""
import pytest

import miters
import oracle
import paper_2512_06627_amd as es

pytestmark = pytest.mark.gpu

FIELDS = ("verdict", "cex", "patterns_evaluated", "next_word")


def _same(a, b):
    return {f: a[f] for f in FIELDS} == {f: b[f] for f in FIELDS}


def _oracle_answer(g):
    c = oracle.Circuit(g.to_aag())
    return c.lowest_failure(threads=8)[0]


def _answer(r):
    return r["cex"] if r["verdict"] == es.FASTLEC_NONEQUIVALENT else None


# (generator, expected verdict) in call order: large then smaller, faulty and equivalent.
CASES = [
    ("minterms n=24, lowest failure deep in the space",
     lambda: miters.minterm_miter(24, [0xB2D3E1, 0xC00001, 0xFFFFFF])),
    ("layered n=22, 3000 gates, fault", lambda: miters.layered_cone_miter(9101, 22, 3000, fault_seed=5)),
    ("mult6 array vs Wallace, fault", lambda: miters.workload("mult6_array_wallace_f1")),
    ("layered n=20, 2500 gates, equivalent", lambda: miters.layered_cone_miter(9102, 20, 2500)),
    ("mult6 array vs Wallace, equivalent", lambda: miters.workload("mult6_array_wallace")),
]


def test_noalloc_matches_plain_check_on_consecutive_calls():
    import torch
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    for label, make in CASES:
        g = make()
        c = es.fastlec_es_load_aig(g.to_aig())
        want = _oracle_answer(g)
        for rep in range(2):  # the same circuit twice: the second call finds the first's contents
            got = es.fastlec_es_check_noalloc(c, stream=stream)
            ref = es.fastlec_es_check(c, kernel="interp", stream=stream)
            assert _same(got, ref), (label, rep, got, ref)
            assert _answer(got) == want, (label, rep, got, want)
            if want is None:
                assert got["patterns_evaluated"] == 1 << c.info()["num_pis"]


def test_noalloc_word_ranges_and_schedules():
    g = miters.workload("mult12_array_booth_f2")
    c = es.fastlec_es_load_aig(g.to_aig())
    full = es.fastlec_es_check(c, kernel="interp")
    assert full["verdict"] == es.FASTLEC_NONEQUIVALENT
    w = full["cex"] // 64
    # a range that starts above the counterexample's word, then one that holds it
    for begin, end in ((w + 1, 1 << 18), (0, w + 1), (w, w + 1)):
        got = es.fastlec_es_check_noalloc(c, begin_word=begin, end_word=end)
        ref = es.fastlec_es_check(c, kernel="interp", begin_word=begin, end_word=end)
        assert _same(got, ref), (begin, end, got, ref)
    for k, wg in ((1, 64), (2, 64), (1, 256)):
        got = es.fastlec_es_check_noalloc(c, words_per_thread=k, wg_size=wg)
        assert _same(got, full), (k, wg, got, full)
    # four words per lane in four-wave workgroups: the value files (about 125 rows of 1 KiB per
    # wave) exceed LDS, and there is no device-memory tier here
    with pytest.raises(es.EsError) as ei:
        es.fastlec_es_check_noalloc(c, words_per_thread=4, wg_size=256)
    assert ei.value.code == es.FASTLEC_ERR_INVALID and "LDS" in str(ei.value)


def test_noalloc_rejects_what_it_cannot_run():
    c = es.fastlec_es_load_aig(miters.workload("mult6_array_wallace_f1").to_aig())
    for kw in ({"kernel": "specialized"}, {"kernel": "interp_hbm"}, {"deadline_s": 1.0}):
        with pytest.raises(es.EsError) as ei:
            es.fastlec_es_check_noalloc(c, **kw)
        assert ei.value.code == es.FASTLEC_ERR_INVALID
    # about 90,000 instructions in bundles of 16: above the array's 65,386
    big = es.fastlec_es_load_aig(miters.layered_cone_miter(77, 10, 120000).to_aig())
    with pytest.raises(es.EsError) as ei:
        es.fastlec_es_check_noalloc(big)
    assert ei.value.code == es.FASTLEC_ERR_INVALID and "exceeds" in str(ei.value)
    # the array still serves a normal call after the rejections
    r = es.fastlec_es_check_noalloc(c)
    assert r["verdict"] == es.FASTLEC_NONEQUIVALENT and r["cex"] == _oracle_answer(miters.workload("mult6_array_wallace_f1"))
