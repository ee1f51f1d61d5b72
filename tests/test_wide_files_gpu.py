"""Value files above the register tier (more than 232 rows): the LDS tier on small spaces and the
device-memory tier (one word per lane, one-wave workgroups) on spaces with a pass for every wave
of its launch, chosen by a plain check without options; both pinned to the oracle.

Faulty cones are pinned by re-evaluation at the reported counterexample plus a scan of the prefix
below it; equivalent ones exhaustively where the space is small enough, else by construction plus
2^20 sampled patterns (tests/pinning.py)."""
import pytest

import miters
import paper_2512_06627_amd as es
from pinning import pin

pytestmark = pytest.mark.gpu

# (generator seed, inputs, AND gates, fault seed): files of 240-420 rows; n 16-20 stay in LDS,
# n 22-24 take the device-memory tier (2^17 and more half-words: a pass for each of 2,048 waves)
CASES = [(9201, 16, 14000, None), (9202, 18, 20000, 3), (9203, 20, 16000, None), (9204, 22, 24000, None),
         (9205, 22, 20000, 5), (9206, 23, 19000, 7), (9207, 24, 16000, None)]


@pytest.mark.parametrize("seed,n,gates,fault", CASES)
def test_wide_file_checks_match_oracle(seed, n, gates, fault):
    g = miters.layered_cone_miter(seed, n, gates, fault_seed=fault)
    c = es.fastlec_es_load_aig(g.to_aig())
    assert c.info()["interp_rows"] > 232, c.info()
    answers = {}
    for opts in ({}, {"kernel": "interp"}, {"kernel": "interp_hbm", "words_per_thread": 1, "wg_size": 64},
                 {"kernel": "interp_hbm", "words_per_thread": 2, "wg_size": 128}):
        r = es.fastlec_es_check(c, **opts)
        assert r["verdict"] in (es.FASTLEC_EQUIVALENT, es.FASTLEC_NONEQUIVALENT), (opts, r)
        answers[str(opts)] = r["cex"] if r["verdict"] == es.FASTLEC_NONEQUIVALENT else None
    assert len(set(answers.values())) == 1, answers
    answer = next(iter(answers.values()))
    assert (answer is not None) == (fault is not None), answers
    pin(g.to_aag(), answer, fault is not None, threads=16, seed=seed)


def test_wide_file_word_ranges_match_oracle():
    # a range that starts just above the first counterexample: its answer is the lowest failing
    # pattern inside the range, or none; the oracle scans the same range
    import oracle
    g = miters.layered_cone_miter(9208, 22, 18000, fault_seed=11)
    c = es.fastlec_es_load_aig(g.to_aig())
    full = es.fastlec_es_check(c)
    assert full["verdict"] == es.FASTLEC_NONEQUIVALENT
    pin(g.to_aag(), full["cex"], True, threads=16, seed=1)
    lo_w = full["cex"] // 64 + 1
    hi_w = lo_w + 4096
    r = es.fastlec_es_check(c, begin_word=lo_w, end_word=hi_w)
    got = r["cex"] if r["verdict"] == es.FASTLEC_NONEQUIVALENT else None
    want, _ = oracle.Circuit(g.to_aag()).lowest_failure(64 * lo_w, 64 * hi_w, threads=16)
    assert got == want, (got, want)
