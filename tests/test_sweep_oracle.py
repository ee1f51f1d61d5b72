"""Pins of the virtual-sweeping oracle (oracle/sweep.py) against facts outside it.

Sources of truth:
  * a hand-worked example (tests/golden/sweep): classes, first-pattern
    polarities and the sub-miter texts of all three targets, derived by hand
    from truth tables;
  * soundness of merging: when the classes come from simulating every pattern
    they are true equivalences (up to complement), so merging a node into its
    representative preserves every function and each target equals its
    representative with its phase: every sub-miter is EQUIVALENT (checked with
    the pinned exact-simulation oracle);
  * faulty miters keep the theorem (classes are still exact), and a class
    built from too few patterns can be wrong: then some sub-miter fails;
  * each sub-miter is a well-formed AIG read by the exact-simulation oracle's
    own reader, on at most as many inputs as the circuit.
Planted mistakes at the end check that the pins can fail.
"""
import json
import os

import numpy as np
import pytest

import miters
import oracle
from oracle import rsim, sweep

HERE = os.path.dirname(__file__)
GOLD = os.path.join(HERE, "golden", "sweep")


def exhaustive_words(n):
    P = 1 << n
    p = np.arange(max(P, 32), dtype=np.uint64) % np.uint64(P)
    rows = []
    for i in range(n):
        bits = ((p >> np.uint64(i)) & np.uint64(1)).astype(np.uint32).reshape(-1, 32)
        rows.append((bits << np.arange(32, dtype=np.uint32)).sum(axis=1, dtype=np.uint32))
    return np.array(rows, dtype=np.uint32).reshape(n, -1)


def classes_and_polarity(aag, words):
    sig = rsim.simulate(aag, words)
    h, _ = rsim.signature_hash(sig)
    return rsim.classes(h).tolist(), (sig[:, 0] & 1).astype(int).tolist()


def test_hand_worked_example():
    spec = json.load(open(os.path.join(GOLD, "spec.json")))
    aag = open(os.path.join(GOLD, spec["circuit"]), "rb").read()
    cls, pol = classes_and_polarity(aag, exhaustive_words(2))
    assert cls == spec["class_of"]
    assert pol == spec["polarity"]
    assert sweep.targets(cls, 2) == sorted(int(t) for t in spec["targets"])
    for t, e in spec["targets"].items():
        text, inputs = sweep.submiter_aag(aag, cls, pol, int(t))
        assert text == open(os.path.join(GOLD, e["file"]), "rb").read(), t
        assert inputs == e["inputs"]
        assert oracle.check(text) is None


CIRCUITS = {
    "mult6_array_wallace": lambda: miters.workload("mult6_array_wallace"),
    "mult6_array_wallace_f1": lambda: miters.workload("mult6_array_wallace_f1"),
    "layered_n10": lambda: miters.layered_cone_miter(3, 10, 600),
    "layered_n10_faulty": lambda: miters.layered_cone_miter(3, 10, 600, fault_seed=5),
}


@pytest.mark.parametrize("name", sorted(CIRCUITS))
def test_exact_classes_give_equivalent_submiters(name):
    g = CIRCUITS[name]()
    aag = g.to_aag()
    cls, pol = classes_and_polarity(aag, exhaustive_words(g.num_inputs))
    ts = sweep.targets(cls, g.num_inputs)
    assert ts, "the circuit should have candidate pairs"
    for t in ts:
        text, inputs = sweep.submiter_aag(aag, cls, pol, t)
        c = oracle.Circuit(text)
        assert c.num_inputs == len(inputs) <= g.num_inputs
        assert inputs == sorted(inputs)
        assert c.lowest_failure()[0] is None, f"target {t}"


def test_partial_simulation_can_propose_false_pairs():
    g = miters.workload("mult6_array_wallace")
    aag = g.to_aag()
    cls, pol = classes_and_polarity(aag, exhaustive_words(g.num_inputs)[:, :1])  # 32 of 4096 patterns
    verdicts = [oracle.check(sweep.submiter_aag(aag, cls, pol, t)[0]) for t in sweep.targets(cls, g.num_inputs)]
    assert any(v is not None for v in verdicts)


def test_rejects_non_targets():
    spec = json.load(open(os.path.join(GOLD, "spec.json")))
    aag = open(os.path.join(GOLD, spec["circuit"]), "rb").read()
    for t in (1, 3, 5, 11):  # an input, representatives, out of range
        with pytest.raises((ValueError, IndexError)):
            sweep.submiter_aag(aag, spec["class_of"], spec["polarity"], t)


# ---- planted mistakes --------------------------------------------------------------

def test_planted_mistakes_are_caught(monkeypatch):
    spec = json.load(open(os.path.join(GOLD, "spec.json")))
    # no phase on merged literals: target 9's fan-in var8 becomes var5 instead of NOT var5
    pol_flat = [0] * len(spec["polarity"])
    aag = open(os.path.join(GOLD, spec["circuit"]), "rb").read()
    text, _ = sweep.submiter_aag(aag, spec["class_of"], pol_flat, 9)
    assert text != open(os.path.join(GOLD, "target9_and_10.aag"), "rb").read()
    assert oracle.check(text) is not None  # and the soundness pin would fail
    # no merging at all: target 9 keeps var8's cone, so the golden text differs
    no_merge = list(range(len(spec["class_of"])))
    no_merge[9] = 3
    text, _ = sweep.submiter_aag(aag, no_merge, spec["polarity"], 9)
    assert text != open(os.path.join(GOLD, "target9_and_10.aag"), "rb").read()
