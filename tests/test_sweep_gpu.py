"""End to end on the GPU: simulation -> candidate classes -> sub-miters -> batched exact simulation.

Step (1) of a sweeping flow proposes candidate pairs from simulation and step
(2) checks them locally (paper, Section 2.3); the paper's units are the
sub-miters of a virtual sweeping pass (Section 3.2).  Here the GPU simulates
and hashes, the library groups classes and extracts sub-miters, and one
batched exact-simulation call checks them all.  Every intermediate result and
every verdict is compared with the oracles (oracle/rsim.py, oracle/sweep.py and
the exact-simulation oracle).
"""
import numpy as np
import pytest

import miters
import oracle
from oracle import rsim, sweep

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def es():
    import paper_2512_06627_amd as m
    return m


def exhaustive_words(n):
    P = 1 << n
    p = np.arange(max(P, 32), dtype=np.uint64) % np.uint64(P)
    rows = [(((p >> np.uint64(i)) & np.uint64(1)).astype(np.uint32).reshape(-1, 32)
             << np.arange(32, dtype=np.uint32)).sum(axis=1, dtype=np.uint32) for i in range(n)]
    return np.array(rows, dtype=np.uint32).reshape(n, -1)


def random_words(n, W, seed):
    r = miters.SplitMix64(seed)
    return np.array([[r.next_u64() & 0xFFFFFFFF for _ in range(W)] for _ in range(n)], dtype=np.uint32).reshape(n, W)


def gpu_classes(g, words):
    E = es()
    c = E.fastlec_es_load_aig(g.to_aig())
    info = c.info()
    n, W = words.shape
    V = info["num_pis"] + info["num_ands"]
    sig = torch.empty((V + 1, W), dtype=torch.int32, device="cuda")
    st = torch.cuda.current_stream()  # the stream torch fills its buffers on
    E.fastlec_es_simulate(c, torch.from_numpy(words.view(np.int32).copy()).cuda(), W, sig, stream=st)
    h = torch.empty(V + 1, dtype=torch.int64, device="cuda")
    ones = torch.empty(V + 1, dtype=torch.int64, device="cuda")
    E.fastlec_es_signature_hash(sig, V + 1, W, h, ones, stream=st)
    cls = E.fastlec_es_classes(h.cpu().numpy().view(np.uint64))
    pol = (sig[:, 0] & 1).to(torch.uint8).cpu().numpy()
    return c, cls, pol


def sweep_on_gpu(g, words, max_inputs=64):
    E = es()
    c, cls, pol = gpu_classes(g, words)
    ocls_sig = rsim.simulate(g.to_aag(), words)
    oh, _ = rsim.signature_hash(ocls_sig)
    want_cls, want_pol = rsim.classes(oh), (ocls_sig[:, 0] & 1).astype(np.uint8)
    assert np.array_equal(cls, want_cls)
    assert np.array_equal(pol, want_pol)
    ts = sweep.targets(cls.tolist(), g.num_inputs)
    subs = [E.fastlec_es_submiter_aag(c, cls, pol, t) for t in ts]
    keep = [i for i, s in enumerate(subs) if len(s[1]) <= max_inputs]
    ts, subs = [ts[i] for i in keep], [subs[i] for i in keep]
    circuits = [E.fastlec_es_load_aig(text) for text, _ in subs]
    results = E.fastlec_es_check_batch(circuits) if circuits else []
    return ts, subs, results


def test_exhaustive_classes_all_submiters_equivalent():
    g = miters.workload("mult6_array_wallace")
    ts, subs, results = sweep_on_gpu(g, exhaustive_words(g.num_inputs))
    assert len(ts) > 10
    assert all(r["verdict"] == es().FASTLEC_EQUIVALENT for r in results)
    for (text, _), r in zip(subs, results):
        assert r["patterns_evaluated"] == 1 << oracle.Circuit(text).num_inputs


@pytest.mark.parametrize("name,make,W,seed", [
    ("mult8_booth_256_patterns", lambda: miters.mult_miter(8, "booth"), 8, 3),
    ("layered_n14", lambda: miters.layered_cone_miter(21, 14, 1200), 2, 5),
    ("mult6_f1_32_patterns", lambda: miters.workload("mult6_array_wallace_f1"), 1, 7),
])
def test_partial_simulation_verdicts_match_oracle(name, make, W, seed):
    g = make()
    ts, subs, results = sweep_on_gpu(g, random_words(g.num_inputs, W, seed))
    assert ts
    for t, (text, _), r in zip(ts, subs, results):
        want = oracle.check(text, threads=8)
        if want is None:
            assert r["verdict"] == es().FASTLEC_EQUIVALENT, f"{name} target {t}"
        else:
            assert r["verdict"] == es().FASTLEC_NONEQUIVALENT and r["cex"] == want, f"{name} target {t}"


def test_full_size_miter_sampled_targets():
    """16x16 multiplier miter, 2^12 random words (2^17 patterns): classes and polarities equal
    the oracle's; the sub-miters on at most 24 inputs run in one batch, and a sample of those on
    at most 20 inputs is checked against the oracle."""
    g = miters.workload("mult16_array_booth")
    words = random_words(32, 1 << 12, seed=16)
    ts, subs, results = sweep_on_gpu(g, words, max_inputs=24)
    assert len(ts) > 20
    small = [(t, s, r) for t, s, r in zip(ts, subs, results) if len(s[1]) <= 20]
    rng = np.random.default_rng(2)
    pick = rng.choice(len(small), min(25, len(small)), replace=False)
    for i in pick:
        t, (text, _), r = small[i]
        want = oracle.check(text, threads=8)
        assert (r["verdict"] == es().FASTLEC_EQUIVALENT) == (want is None), t
        if want is not None:
            assert r["cex"] == want
