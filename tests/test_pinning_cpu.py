"""The pinning rule of tests/pinning.py, checked on the CPU against answers the oracle or the
construction fixes, and against planted wrong answers, each of which it must reject."""
import pytest

import miters
import oracle
from pinning import pin, sample_windows


def test_sample_windows_cover_ends_and_are_disjoint():
    for n, sample, w in ((20, 1 << 12, 1 << 8), (34, 1 << 20, 1 << 16), (10, 1 << 12, 1 << 8)):
        ws = sample_windows(n, seed=3, sample=sample, window=w)
        assert ws[0][0] == 0 and ws[-1][1] == 1 << n
        assert all(a[1] <= b[0] for a, b in zip(ws, ws[1:]))
        assert sum(hi - lo for lo, hi in ws) == min(sample, 1 << n)


def _faulty():
    g = miters.workload("mult6_array_wallace_f1")
    return g.to_aag(), oracle.check(g.to_aag())


def test_correct_answers_are_pinned():
    aag, cex = _faulty()
    assert cex is not None and cex > 0
    assert pin(aag, cex, True, threads=4) == "cex+prefix"
    assert pin(aag, cex, True, threads=4, exhaustive_budget=1) == "cex+sampled prefix"
    eq = miters.workload("mult6_array_wallace").to_aag()
    assert pin(eq, None, False, threads=4) == "exhaustive"
    cone = miters.layered_cone_miter(31, 14, 600).to_aag()
    assert pin(cone, None, False, threads=4, exhaustive_budget=1, sample=1 << 10) == "construction+sampled"


def test_planted_wrong_answers_are_rejected():
    aag, cex = _faulty()
    c = oracle.Circuit(aag)
    above = next(p for p in range(cex + 1, 1 << 12) if c.miter([p])[0] == 1)
    clean = next(p for p in range(cex + 1, 1 << 12) if c.miter([p])[0] == 0)
    for wrong in (above, clean):  # a higher failing pattern; a pattern that does not fail
        with pytest.raises(AssertionError):
            pin(aag, wrong, True, threads=4)
    with pytest.raises(AssertionError):  # EQUIVALENT claimed within the exhaustive budget
        pin(aag, None, True, threads=4)
    with pytest.raises(AssertionError):  # above the budget, an injected fault is not pinned by sampling
        pin(aag, None, True, threads=4, exhaustive_budget=1)
    # above the budget, sampling still catches a failure in the always-scanned first window
    low = miters.minterm_miter(16, [5]).to_aag()
    with pytest.raises(AssertionError):
        pin(low, None, False, threads=4, exhaustive_budget=1, sample=1 << 10)
