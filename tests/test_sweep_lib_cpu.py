"""The library's sub-miter extraction (host code) against the virtual-sweeping oracle.

fastlec_es_submiter_aag runs on the host, so its parity with oracle/sweep.py is
checked here without a GPU: byte-identical AIGER text and the same input map
for every target of several circuits, with classes from exhaustive and from
partial simulation (oracle/rsim.py supplies them; both sides get the same).
"""
import json
import os

import numpy as np
import pytest

import miters
import paper_2512_06627_amd as es
from oracle import rsim, sweep

GOLD = os.path.join(os.path.dirname(__file__), "golden", "sweep")


def words_for(n, W, seed):
    r = miters.SplitMix64(seed)
    return np.array([[r.next_u64() & 0xFFFFFFFF for _ in range(W)] for _ in range(n)], dtype=np.uint32).reshape(n, W)


def exhaustive_words(n):
    P = 1 << n
    p = np.arange(max(P, 32), dtype=np.uint64) % np.uint64(P)
    rows = [(((p >> np.uint64(i)) & np.uint64(1)).astype(np.uint32).reshape(-1, 32)
             << np.arange(32, dtype=np.uint32)).sum(axis=1, dtype=np.uint32) for i in range(n)]
    return np.array(rows, dtype=np.uint32).reshape(n, -1)


def classes_and_polarity(aag, words):
    sig = rsim.simulate(aag, words)
    h, _ = rsim.signature_hash(sig)
    return rsim.classes(h), (sig[:, 0] & 1).astype(np.uint8)


def test_golden_example():
    spec = json.load(open(os.path.join(GOLD, "spec.json")))
    aag = open(os.path.join(GOLD, spec["circuit"]), "rb").read()
    c = es.fastlec_es_load_aig(aag)
    for t, e in spec["targets"].items():
        text, inputs = es.fastlec_es_submiter_aag(c, spec["class_of"], spec["polarity"], int(t))
        assert text == open(os.path.join(GOLD, e["file"]), "rb").read()
        assert inputs == e["inputs"]


CASES = [
    ("mult6_exhaustive", lambda: miters.workload("mult6_array_wallace"), None),
    ("mult6_f1_32_patterns", lambda: miters.workload("mult6_array_wallace_f1"), 1),
    ("mult8_array_booth_random", lambda: miters.mult_miter(8, "booth"), 8),
    ("layered_n16_random", lambda: miters.layered_cone_miter(9, 16, 1500), 4),
    ("mac4_random", lambda: miters.mac_miter(4), 2),
]


@pytest.mark.parametrize("name,make,W", CASES, ids=[c[0] for c in CASES])
def test_every_target_matches_oracle(name, make, W):
    g = make()
    aag = g.to_aag()
    words = exhaustive_words(g.num_inputs) if W is None else words_for(g.num_inputs, W, seed=W)
    cls, pol = classes_and_polarity(aag, words)
    c = es.fastlec_es_load_aig(g.to_aig())
    ts = sweep.targets(cls.tolist(), g.num_inputs)
    assert ts
    for t in ts:
        want = sweep.submiter_aag(aag, cls.tolist(), pol.tolist(), t)
        got = es.fastlec_es_submiter_aag(c, cls, pol, t)
        assert got[0] == want[0], f"{name} target {t}"
        assert got[1] == want[1]


def test_errors():
    spec = json.load(open(os.path.join(GOLD, "spec.json")))
    c = es.fastlec_es_load_aig(open(os.path.join(GOLD, spec["circuit"]), "rb").read())
    cls, pol = spec["class_of"], spec["polarity"]
    for t in (1, 3, 5, 11, 0):
        with pytest.raises(es.EsError) as ei:
            es.fastlec_es_submiter_aag(c, cls, pol, t)
        assert ei.value.code == -5
    with pytest.raises(es.EsError):
        es.fastlec_es_submiter_aag(c, cls[:-1], pol[:-1], 8)          # wrong length
    with pytest.raises(es.EsError):
        es.fastlec_es_submiter_aag(c, cls, [2] * len(pol), 8)          # polarity not 0/1
    bad = list(cls)
    bad[6] = 7                                                          # representative above member
    bad[8] = 6
    with pytest.raises(es.EsError):
        es.fastlec_es_submiter_aag(c, bad, pol, 8)


def test_representatives_that_are_inputs_or_constants():
    """pi_and_const.aag: var4 = a & ~(~a & ~b) equals input a, var5 = a & ~a is constant false,
    var6 = var4 & ~var5 equals a.  Sub-miters then hold input and constant literals; the library
    writes the oracle's text and every sub-miter is equivalent (the classes are exact)."""
    import oracle
    text = open(os.path.join(GOLD, "pi_and_const.aag"), "rb").read()
    cls, pol = classes_and_polarity(text, exhaustive_words(2))
    assert cls.tolist() == [0, 1, 2, 3, 1, 0, 1]
    c = es.fastlec_es_load_aig(text)
    ts = sweep.targets(cls.tolist(), 2)
    assert ts == [4, 5, 6]
    for t in ts:
        want = sweep.submiter_aag(text, cls.tolist(), pol.tolist(), t)
        got = es.fastlec_es_submiter_aag(c, cls, pol, t)
        assert got == want
        assert oracle.check(got[0]) is None
    # the constant target's sub-miter reads only constants and input a
    assert sweep.submiter_aag(text, cls.tolist(), pol.tolist(), 5)[1] == [0]
