"""Pins of the plain CPU oracle against facts fixed outside the oracle.

Each pin is chosen so that a plausible slip in the oracle (a dropped
complement, a wrong input-bit mapping, a lost output, a scan that does not
return the minimum, an off-by-one range) fails at least one test; the
mutation test in test_oracle_mutants.py checks exactly that.

Sources of truth:
  * closed-form arithmetic: a*b and a*b + c*d, exhaustive at small widths
    (this also pins the seeded generators);
  * hand-worked miters in tests/golden/hand (paper, Section 2.1 miter
    definition; Section 2.2 exact simulation);
  * minterm circuits whose failing set is known by construction;
  * cost_ES = 2^num_PIs (paper, Section 3.2 feature iii): an equivalent miter
    is proved after exactly 2^n patterns.
"""
import json
import os

import numpy as np
import pytest

import miters
import oracle
from miters.miter import mult_circuit, mac_circuit

pytestmark = pytest.mark.filterwarnings("ignore")


def products(ps, w):
    a = ps & np.uint64((1 << w) - 1)
    b = ps >> np.uint64(w)
    return a * b


def mac_values(ps, w):
    m = np.uint64((1 << w) - 1)
    a, b = ps & m, (ps >> np.uint64(w)) & m
    c, d = (ps >> np.uint64(2 * w)) & m, (ps >> np.uint64(3 * w)) & m
    return a * b + c * d


# ---- hand-worked fixtures -------------------------------------------------

def _hand_cases():
    path = os.path.join(os.path.dirname(__file__), "golden", "hand_worked.json")
    spec = json.load(open(path))
    return [(k, v) for k, v in spec.items() if not k.startswith("_")]


@pytest.mark.parametrize("name,spec", _hand_cases(), ids=[k for k, _ in _hand_cases()])
def test_hand_worked(name, spec, golden_dir):
    text = open(os.path.join(golden_dir, "hand", name), "rb").read()
    if "error" in spec:
        with pytest.raises(oracle.OracleError) as ei:
            oracle.check(text)
        assert ei.value.code == {"parse": -1, "unsupported": -2}[spec["error"]]
    else:
        c = oracle.Circuit(text)
        p, evaluated = c.lowest_failure()
        assert p == spec["expect"]
        if p is None:
            assert evaluated == 1 << c.num_inputs


# ---- closed-form arithmetic ---------------------------------------------------

@pytest.mark.parametrize("kind", ["array", "wallace", "booth"])
@pytest.mark.parametrize("w", [1, 2, 3, 4, 5, 6, 7])
def test_multiplier_closed_form(kind, w):
    c = oracle.Circuit(mult_circuit(kind, w).to_aag())
    assert c.num_inputs == 2 * w and c.num_outputs == 2 * w
    ps = np.arange(1 << (2 * w), dtype=np.uint64)
    assert np.array_equal(c.outputs(ps), products(ps, w))


@pytest.mark.parametrize("kind", ["fused", "separate"])
@pytest.mark.parametrize("w", [1, 2, 3, 4])
def test_mac_closed_form(kind, w):
    c = oracle.Circuit(mac_circuit(kind, w).to_aag())
    assert c.num_inputs == 4 * w and c.num_outputs == 2 * w + 1
    ps = np.arange(1 << (4 * w), dtype=np.uint64)
    assert np.array_equal(c.outputs(ps), mac_values(ps, w))


@pytest.mark.parametrize("kind", ["array", "booth"])
def test_multiplier_closed_form_sampled_16(kind):
    """16x16 products on 4096 seeded random patterns (exhaustive is 2^32)."""
    rng = miters.SplitMix64(16)
    ps = np.array([rng.next_u64() >> 32 for _ in range(4096)] + [0, (1 << 32) - 1], dtype=np.uint64)
    c = oracle.Circuit(mult_circuit(kind, 16).to_aag())
    assert np.array_equal(c.outputs(ps), products(ps, 16))


def test_mac8_closed_form_sampled():
    rng = miters.SplitMix64(8)
    ps = np.array([rng.next_u64() >> 32 for _ in range(4096)] + [0, (1 << 32) - 1], dtype=np.uint64)
    for kind in ("fused", "separate"):
        c = oracle.Circuit(mac_circuit(kind, 8).to_aag())
        assert np.array_equal(c.outputs(ps), mac_values(ps, 8))


# ---- miters ---------------------------------------------------------------

@pytest.mark.parametrize("impl", ["wallace", "booth"])
@pytest.mark.parametrize("w", [2, 4, 6])
def test_equivalent_miter_costs_2_pow_n(impl, w):
    """An equivalent miter is proved only after all 2^n patterns (cost_ES = 2^num_PIs)."""
    c = oracle.Circuit(miters.mult_miter(w, impl).to_aag())
    p, evaluated = c.lowest_failure(threads=3)
    assert p is None and evaluated == 1 << (2 * w)


@pytest.mark.parametrize("seed", range(1, 9))
@pytest.mark.parametrize("impl,w", [("wallace", 5), ("booth", 6)])
def test_faulty_multiplier_lowest_cex_by_closed_form(impl, w, seed):
    """Lowest counterexample of a faulted multiplier miter, checked against a*b.

    The reference side is the array multiplier, pinned to a*b above, so the
    miter fails at p iff the faulted circuit's output differs from a*b at p.
    """
    spec, bad = miters.mult_pair(w, impl, fault_seed=seed)
    p = oracle.check(miters.miter_of(spec, bad).to_aag(), threads=4)
    ps = np.arange(1 << (2 * w), dtype=np.uint64)
    wrong = np.nonzero(oracle.Circuit(bad.to_aag()).outputs(ps) != products(ps, w))[0]
    assert p == (int(wrong[0]) if wrong.size else None)


def test_faulty_mac_lowest_cex_by_closed_form():
    for seed in (1, 2, 3):
        spec = mac_circuit("separate", 3)
        bad = miters.inject_fault(mac_circuit("fused", 3), seed)
        p = oracle.check(miters.miter_of(spec, bad).to_aag(), threads=4)
        ps = np.arange(1 << 12, dtype=np.uint64)
        wrong = np.nonzero(oracle.Circuit(bad.to_aag()).outputs(ps) != mac_values(ps, 3))[0]
        assert p == (int(wrong[0]) if wrong.size else None)


def test_multi_output_miter_matches_or_of_outputs():
    """A miter kept as one XOR per output pair fails exactly where the OR-reduced one does."""
    spec, bad = miters.mult_pair(4, "booth", fault_seed=5)
    single = miters.miter_of(spec, bad, or_outputs=True)
    multi = miters.miter_of(spec, bad, or_outputs=False)
    assert len(multi.outputs) == 8
    ps = np.arange(256, dtype=np.uint64)
    want = (oracle.Circuit(bad.to_aag()).outputs(ps) != products(ps, 4)).astype(np.uint8)
    assert np.array_equal(oracle.Circuit(single.to_aag()).miter(ps), want)
    assert np.array_equal(oracle.Circuit(multi.to_aag()).miter(ps), want)


# ---- minterm circuits ---------------------------------------------------------

@pytest.mark.parametrize("n,targets", [
    (1, [1]), (3, [5]), (6, [63]), (7, [64]), (8, [200, 17]), (10, [1023]),
    (12, [2048, 4095, 777]), (16, [65535]), (16, [1 << 15, 12345, 54321]), (20, [999_999, 1 << 19]),
])
def test_minterm_lowest(n, targets):
    c = oracle.Circuit(miters.minterm_miter(n, targets).to_aag())
    p, evaluated = c.lowest_failure(threads=4)
    assert p == min(targets)


def test_minterm_failing_set_exact():
    rng = miters.SplitMix64(7)
    n = 11
    targets = sorted({rng.below(1 << n) for _ in range(9)})
    c = oracle.Circuit(miters.minterm_miter(n, targets).to_aag())
    ps = np.arange(1 << n, dtype=np.uint64)
    assert list(np.nonzero(c.miter(ps))[0]) == targets


def test_scan_ranges_and_threads():
    targets = [100, 5000, 70000, 1 << 19]
    c = oracle.Circuit(miters.minterm_miter(20, targets).to_aag())
    for threads in (1, 2, 3, 8):
        assert c.lowest_failure(threads=threads)[0] == 100
        assert c.lowest_failure(101, threads=threads)[0] == 5000
        assert c.lowest_failure(5000, 5001, threads=threads)[0] == 5000
        assert c.lowest_failure(5001, 70000, threads=threads)[0] is None
        assert c.lowest_failure(70001, threads=threads)[0] == 1 << 19
        assert c.lowest_failure(0, 0, threads=threads)[0] is None


def test_aiger_binary_is_not_read_by_oracle():
    """The oracle only reads ASCII AIGER; binary files are a GPU-path feature pinned against it."""
    with pytest.raises(oracle.OracleError):
        oracle.Circuit(miters.mult_miter(2, "booth").to_aig())
