"""Pinning GPU answers on cones whose full pattern space is too large for the oracle.

Exact simulation has a plain definition (paper, Section 2.1 miter; Section 2.2 exact
simulation): the answer is the lowest pattern p whose miter output is 1, or none.  For a
cone of n inputs and N gates the oracle's full scan costs 2^n * N gate evaluations, so each
answer is pinned by the cheapest check that still fixes it:

* a reported counterexample p is re-evaluated (the miter must be 1 at p: soundness) and the
  prefix [0, p) is scanned (no failure below p: minimality).  This fixes the answer exactly
  and costs p * N, small for the seeded faults here;
* EQUIVALENT on a space of at most ``exhaustive_budget`` gate evaluations is pinned by the
  full scan;
* EQUIVALENT above that budget is pinned by equivalence by construction (a cone without an
  injected fault is equivalent because every cell rewrite of its generator is exhaustively
  verified in test_generators.py) plus a scan of seeded windows that together hold
  ``sample`` patterns, the first and last window included.

``pin`` returns the method used, so tests and reports can count them.
"""
import oracle
from miters import SplitMix64

EXHAUSTIVE_BUDGET = 1 << 33
SAMPLE = 1 << 20
WINDOW = 1 << 16


def sample_windows(n: int, seed: int, sample: int = SAMPLE, window: int = WINDOW):
    """Ascending disjoint windows [s, s + w) of [0, 2^n) holding `sample` patterns."""
    space = 1 << n
    if sample >= space:
        return [(0, space)]
    w = min(window, sample)
    slots = space // w
    k = max(2, sample // w)
    rng = SplitMix64(seed)
    chosen = {0, slots - 1}
    while len(chosen) < k:
        chosen.add(rng.below(slots))
    return [(s * w, s * w + w) for s in sorted(chosen)]


def pin(aag: bytes, answer, injected: bool, threads: int, seed: int = 0,
        exhaustive_budget: int = EXHAUSTIVE_BUDGET, sample: int = SAMPLE) -> str:
    """Check a GPU answer (lowest failing pattern or None) against the oracle; returns the method
    ("cex+prefix", "cex+sampled prefix", "exhaustive", "construction+sampled").  Raises
    AssertionError when the answer is wrong."""
    c = oracle.Circuit(aag)
    n, gates = c.num_inputs, max(1, c.num_ands)
    if answer is not None:
        assert 0 <= answer < (1 << n), answer
        assert c.miter([answer])[0] == 1, f"miter is 0 at the reported counterexample {answer}"
        if answer * gates <= exhaustive_budget:
            p, _ = c.lowest_failure(0, answer, threads=threads)
            assert p is None, f"lower failing pattern {p} below the reported {answer}"
            return "cex+prefix"
        for lo, hi in sample_windows(max(1, answer.bit_length()), seed, sample):
            lo, hi = min(lo, answer), min(hi, answer)
            if lo < hi:
                p, _ = c.lowest_failure(lo, hi, threads=threads)
                assert p is None, f"lower failing pattern {p} below the reported {answer}"
        return "cex+sampled prefix"
    if (1 << n) * gates <= exhaustive_budget:
        p, _ = c.lowest_failure(threads=threads)
        assert p is None, f"the oracle finds failing pattern {p}"
        return "exhaustive"
    assert not injected, "an injected fault answered EQUIVALENT above the exhaustive budget is not pinned"
    for lo, hi in sample_windows(n, seed, sample):
        p, _ = c.lowest_failure(lo, hi, threads=threads)
        assert p is None, f"the oracle finds failing pattern {p} in [{lo}, {hi})"
    return "construction+sampled"
