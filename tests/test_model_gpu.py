"""The runtime model against measured kernel times, and the batch's use of it.

The paper predicts ES time from the gate and input counts with coefficients fitted
on measurements (Section 3.2, runtime prediction) and uses the prediction to pick
engines.  The library fits that form per kernel on MI355X (paper_2512_06627_amd/
calibrate.py); here held-out cones (other seeds, sizes and input counts than the
fitting set) must be predicted within a factor of two, and a batch must send the
cones the model favours to the specialized kernel with answers equal to the oracle's.
"""
import pytest

import miters
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def es():
    import paper_2512_06627_amd as m
    return m


HELD_OUT = [(5, 21, 2500), (6, 23, 700), (7, 25, 4000), (8, 27, 1500), (9, 19, 6000)]


@pytest.mark.parametrize("seed,n,gates", HELD_OUT)
def test_predictions_within_factor_two(seed, n, gates):
    E = es()
    c = E.fastlec_es_load_aig(miters.layered_cone_miter(seed, n, gates).to_aig())
    p = E.fastlec_es_predict(c)
    for kern in ("interp", "specialized"):
        r = E.fastlec_es_check(c, kernel=kern)
        if kern == "specialized":
            assert 0.5 < p["compile_ms"] / max(r["compile_ms"], 1e-3) < 2.0 or r["compile_ms"] == 0
        ms = sorted(E.fastlec_es_check(c, kernel=kern)["kernel_ms"] for _ in range(5))[2]
        assert 0.5 < p[kern + "_ms"] / ms < 2.0, (kern, p[kern + "_ms"], ms)


def test_batch_routes_large_cones_to_specialized_kernel():
    E = es()
    gs = [miters.layered_cone_miter(60 + i, 14 + i % 3, 300) for i in range(6)]
    gs += [miters.mult_miter(12, "booth"), miters.mult_miter(12, "booth", fault_seed=3),
           miters.layered_cone_miter(72, 33, 6000), miters.layered_cone_miter(73, 33, 4000, fault_seed=2)]
    cs = [E.fastlec_es_load_aig(g.to_aig()) for g in gs]
    res = E.fastlec_es_check_batch(cs)
    want_spec = []
    for c in cs:
        p = E.fastlec_es_predict(c)
        want_spec.append(p["specialized_ms"] + 1.2 * p["compile_ms"] < p["interp_ms"])
    assert any(want_spec) and not all(want_spec)
    for g, c, r, ws in zip(gs, cs, res, want_spec):
        # a routed cone's kernel is compiled already; compiling again costs nothing
        if ws:
            assert E.fastlec_es_compile_specialized(c, 3)["compile_ms"] == 0
        if g.num_inputs <= 24:
            want = oracle.check(g.to_aag(), threads=16)
            assert (r["verdict"] == E.FASTLEC_EQUIVALENT) == (want is None)
            if want is not None:
                assert r["cex"] == want
        alone = E.fastlec_es_check(c, kernel="interp")
        assert (r["verdict"], r["cex"]) == (alone["verdict"], alone["cex"])


def test_kernels_compiled_together_give_oracle_answers():
    """Kernels from one multi-kernel hipRTC program, launched by their own entry points."""
    E = es()
    gs = [miters.layered_cone_miter(90 + i, 16 + i % 4, 800, fault_seed=(i if i % 2 else None)) for i in range(8)]
    cs = [E.fastlec_es_load_aig(g.to_aig()) for g in gs]
    assert E.fastlec_es_compile_specialized_many(cs, 3) > 0
    for g, c in zip(gs, cs):
        r = E.fastlec_es_check(c, kernel="specialized")
        assert r["compile_ms"] == 0
        want = oracle.check(g.to_aag(), threads=16)
        assert (r["verdict"] == E.FASTLEC_EQUIVALENT) == (want is None)
        if want is not None:
            assert r["cex"] == want


def test_batch_runs_large_interpreter_cones_alone():
    """With the interpreter forced, cones predicted at 1 ms or more run as their own launches and
    the rest share grouped launches; every answer equals the cone checked alone (and the
    oracle's for the small ones), and the large cones report their own kernel times."""
    E = es()
    small = [miters.layered_cone_miter(120 + i, 12 + i % 5, 400, fault_seed=(i if i % 2 else None)) for i in range(6)]
    large = [miters.layered_cone_miter(130 + i, 27 + i % 2, 3000, fault_seed=(7 if i == 1 else None)) for i in range(3)]
    gs = small + large
    cs = [E.fastlec_es_load_aig(g.to_aig()) for g in gs]
    preds = [E.fastlec_es_predict(c)["interp_ms"] for c in cs]
    assert all(p < 1.0 for p in preds[:6]) and all(p >= 1.0 for p in preds[6:])
    res = E.fastlec_es_check_batch(cs, kernel="interp")
    for g, c, r in zip(gs, cs, res):
        alone = E.fastlec_es_check(c, kernel="interp")
        assert (r["verdict"], r["cex"]) == (alone["verdict"], alone["cex"])
        if g.num_inputs <= 16:
            want = oracle.check(g.to_aag(), threads=16)
            assert (r["cex"] if r["verdict"] else None) == want
    grouped_ms = {r["kernel_ms"] for r in res[:6]}
    assert len(grouped_ms) == 1                      # one sum over the grouped launches
    assert all(r["kernel_ms"] not in grouped_ms for r in res[6:])
