"""The batched and serving workloads at their stated sizes, every answer pinned by the oracle.

Batch: the 256 layered cones of the batched-ES workload (n 18..30 inputs, about 200..5000 AND
gates, 26 with an injected fault; the same seeded set the benchmark's batch leg runs), checked
by one batched call with the runtime model's routing (specialized kernels for the large cones)
and by one on the interpreter alone.  Serve: the 40-cone pool of the serving workload (n 16..34,
about 500..20000 gates, 10% faulty), all submitted to one server at once.

Each answer is pinned by tests/pinning.py: a counterexample by re-evaluation at it and a scan of
the prefix below it; EQUIVALENT by the full scan where 2^n * N <= 2^33 gate evaluations, else by
equivalence by construction plus 2^20 oracle-scanned patterns in seeded windows.  The counts per
method are printed (run with -s to see them).
"""
import os
from collections import Counter

import pytest

import miters
import oracle
import paper_2512_06627_amd as es
from pinning import pin

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, len(os.sched_getaffinity(0))))
CHUNKS = 8
_counts = {"batch": Counter(), "serve": Counter()}


def _answers(rs):
    out = []
    for r in rs:
        assert r["verdict"] in (es.FASTLEC_EQUIVALENT, es.FASTLEC_NONEQUIVALENT), r
        out.append(r["cex"] if r["verdict"] == es.FASTLEC_NONEQUIVALENT else None)
    return out


@pytest.fixture(scope="module")
def batch_run():
    items = miters.cone_batch(4, 256, 26, (18, 30), (200, 5000))
    cones = [es.fastlec_es_load_aig(g.to_aig()) for g, _ in items]
    print("batch workload loaded", flush=True)
    routed = _answers(es.fastlec_es_check_batch(cones))
    print("batch with the model's routing done", flush=True)
    interp = _answers(es.fastlec_es_check_batch(cones, kernel="interp"))
    print("batch on the interpreter done", flush=True)
    assert routed == interp
    return items, routed


@pytest.mark.parametrize("chunk", range(CHUNKS))
def test_batch_workload_pinned_by_oracle(batch_run, chunk):
    items, ans = batch_run
    for i in range(chunk, len(items), CHUNKS):
        g, fault = items[i]
        if fault is None:
            assert ans[i] is None, (i, ans[i])  # equivalent by construction
        method = pin(g.to_aag(), ans[i], fault is not None, THREADS, seed=i)
        _counts["batch"][method] += 1
    print("batch chunk", chunk, dict(_counts["batch"]), flush=True)


def test_batch_workload_all_pinned():
    c = _counts["batch"]
    print("batch workload pinned:", dict(c), flush=True)
    assert sum(c.values()) == 256
    assert c["cex+prefix"] + c["cex+sampled prefix"] == 26  # every injected fault is visible


@pytest.fixture(scope="module")
def serve_run():
    items = miters.serve_pool(miters.SplitMix64(5), 5, 40)
    circs = [es.fastlec_es_load_aig(g.to_aig()) for g, _ in items]
    print("serving pool loaded", flush=True)
    srv = es.Server(64 << 30)
    try:
        tickets = [srv.submit(c) for c in circs]
        served = _answers([srv.poll(t, wait=True) for t in tickets])
        st = srv.stats()
    finally:
        srv.close()
    print("served", st["completed"], "jobs, at most", st["max_active"], "in flight", flush=True)
    assert st["max_active"] >= 2
    alone = _answers([es.fastlec_es_check(c) for c in circs])
    assert served == alone
    return items, served


@pytest.mark.parametrize("chunk", range(4))
def test_serve_workload_pinned_by_oracle(serve_run, chunk):
    items, ans = serve_run
    for i in range(chunk, len(items), 4):
        g, fault = items[i]
        if fault is None:
            assert ans[i] is None, (i, ans[i])
        method = pin(g.to_aag(), ans[i], fault is not None, THREADS, seed=1000 + i)
        _counts["serve"][method] += 1
    print("serve chunk", chunk, dict(_counts["serve"]), flush=True)


def test_serve_workload_all_pinned():
    c = _counts["serve"]
    print("serving pool pinned:", dict(c), flush=True)
    assert sum(c.values()) == 40


def test_wide_cones_specialized_match_oracle():
    """Cones whose live values exceed the three-wave register budget run at two or one wave per
    SIMD with LDS spills; their answers must equal the oracle's full scan (2^22 patterns)."""
    for size, n in ((12000, 22), (20000, 22)):
        for fault in (None, 5):
            g = miters.layered_cone_miter(900000 + size, n, size, fault_seed=fault)
            c = es.fastlec_es_load_aig(g.to_aig())
            src = es.fastlec_es_specialized_source(c, 3)
            assert "one asm block:" in src and ("2 waves per SIMD" in src or "1 waves per SIMD" in src), size
            if size == 20000:
                assert "LDS spill" in src
            print("wide cone", size, n, fault, flush=True)
            want = oracle.check(g.to_aag(), threads=THREADS)
            for kernel in ("specialized", "interp"):
                r = es.fastlec_es_check(c, kernel=kernel)
                assert _answers([r]) == [want], (size, fault, kernel)
