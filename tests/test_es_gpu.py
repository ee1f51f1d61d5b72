"""GPU parity: the HIP exact-simulation path against the oracle, bit for bit.

Every expected value comes from the oracle (directly, or from
tests/golden/expected.json, written by tests/golden/make_expected.py with the
oracle only) or from the hand-worked fixtures.  The answer compared is the
verdict and the lowest failing pattern, which are unique.
"""
import json
import os

import numpy as np
import pytest

import miters
import oracle
import paper_2512_06627_amd as es

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
KERNELS = ["interp", "interp_hbm", "specialized"]


def expected(name):
    return json.load(open(os.path.join(GOLDEN, "expected.json")))[name]["lowest_failure"]


def gpu_answer(circ, **kw):
    r = es.fastlec_es_check(circ, **kw)
    if r["verdict"] == es.FASTLEC_EQUIVALENT:
        return None
    assert r["verdict"] == es.FASTLEC_NONEQUIVALENT
    return r["cex"]


def hand_cases():
    spec = json.load(open(os.path.join(GOLDEN, "hand_worked.json")))
    return [(k, v) for k, v in spec.items() if not k.startswith("_")]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("name,spec", hand_cases(), ids=[k for k, _ in hand_cases()])
def test_hand_worked(name, spec, kernel):
    data = open(os.path.join(GOLDEN, "hand", name), "rb").read()
    if "error" in spec:
        with pytest.raises(es.EsError) as ei:
            es.fastlec_es_load_aig(data)
        assert ei.value.code == {"parse": es.FASTLEC_ERR_PARSE, "unsupported": es.FASTLEC_ERR_UNSUPPORTED}[spec["error"]]
        return
    c = es.fastlec_es_load_aig(data)
    r = es.fastlec_es_check(c, kernel=kernel)
    assert gpu_answer(c, kernel=kernel) == spec["expect"]
    if spec["expect"] is None:
        n = c.info()["num_pis"]
        assert r["patterns_evaluated"] == 1 << n  # cost_ES = 2^num_PIs


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("name", ["mult6_array_wallace", "mult6_array_wallace_f1", "mult12_array_booth",
                                  "mult12_array_booth_f1", "mult12_array_booth_f2", "mult12_array_booth_f3",
                                  "mult12_array_booth_f4"])
def test_workloads_match_oracle_golden(name, kernel):
    g = miters.workload(name)
    for data in (g.to_aag(), g.to_aig()):
        c = es.fastlec_es_load_aig(data)
        assert gpu_answer(c, kernel=kernel) == expected(name)


@pytest.mark.parametrize("name", ["mult16_array_booth_f1", "mult16_array_booth_f2", "mult16_array_booth_f3",
                                  "mult16_array_booth_f4", "mac8_fused_separate_f1"])
def test_full_size_faults_match_oracle_golden(name):
    exp = expected(name)
    c = es.fastlec_es_load_aig(miters.workload(name).to_aig())
    for kernel in ("specialized", "interp"):
        assert gpu_answer(c, kernel=kernel) == exp


def _minterm_cases():
    cases = []
    for n in (1, 3, 5, 6, 7, 11, 12, 13, 17):
        top = (1 << n) - 1
        for t in sorted({0, 1, 31, 32, 63, 64, 2047, 2048, 4095, 4096, 65535, 65536, top // 2, top - 1, top}):
            if t <= top:
                cases.append((n, (t,)))
    cases += [(20, (999_999, 1 << 19)), (20, (5, 1048575)), (16, (40000, 40001, 39999))]
    return cases


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("n,targets", _minterm_cases())
def test_minterm_edges(n, targets, kernel):
    """A minterm circuit fails exactly at its targets: lowest = min (lane, wave, tile and word edges)."""
    c = es.fastlec_es_load_aig(miters.minterm_miter(n, targets).to_aag())
    assert gpu_answer(c, kernel=kernel) == min(targets)


@pytest.mark.parametrize("K", [1, 2, 4])
@pytest.mark.parametrize("wg", [64, 256])
@pytest.mark.parametrize("tile_words", [0, 32, 1024])
def test_schedule_invariance(K, wg, tile_words):
    for name in ("mult12_array_booth_f2", "mult12_array_booth_f3"):
        c = es.fastlec_es_load_aig(miters.workload(name).to_aig())
        for kernel in ("interp", "interp_hbm"):
            assert gpu_answer(c, kernel=kernel, words_per_thread=K, wg_size=wg, tile_words=tile_words) == expected(name)


def test_word_ranges_resume():
    """Checking [0, a) then [a, W) gives the same answer as one call (resume support)."""
    name = "mult12_array_booth_f1"
    exp = expected(name)
    c = es.fastlec_es_load_aig(miters.workload(name).to_aig())
    W = 1 << 18
    for kernel in KERNELS:
        for a in (1, exp // 64, exp // 64 + 1, W // 2):
            r1 = es.fastlec_es_check(c, kernel=kernel, begin_word=0, end_word=a)
            r2 = es.fastlec_es_check(c, kernel=kernel, begin_word=a, end_word=W)
            first = r1["cex"] if r1["verdict"] else (r2["cex"] if r2["verdict"] else None)
            assert first == exp
            if r1["verdict"] == es.FASTLEC_EQUIVALENT:
                assert r1["patterns_evaluated"] == 64 * a and r1["next_word"] == a


def test_equivalent_range_counts():
    c = es.fastlec_es_load_aig(miters.workload("mult12_array_booth").to_aig())
    for kernel in KERNELS:
        r = es.fastlec_es_check(c, kernel=kernel)
        assert r["verdict"] == es.FASTLEC_EQUIVALENT and r["patterns_evaluated"] == 1 << 24
        assert r["next_word"] == 1 << 18


def test_repeated_runs_deterministic():
    c = es.fastlec_es_load_aig(miters.workload("mult12_array_booth_f4").to_aig())
    got = {gpu_answer(c, kernel=k) for k in KERNELS for _ in range(3)}
    assert got == {expected("mult12_array_booth_f4")}


def test_layered_cones_vs_oracle():
    rng = miters.SplitMix64(77)
    for i in range(8):
        n = rng.between(8, 16)
        fault = rng.between(1, 100) if i % 2 else None
        g = miters.layered_cone_miter(1000 + i, n, rng.between(200, 1500), fault_seed=fault)
        want = oracle.check(g.to_aag(), threads=8)
        c = es.fastlec_es_load_aig(g.to_aig())
        for kernel in KERNELS:
            assert gpu_answer(c, kernel=kernel) == want


def test_batch_matches_single():
    rng = miters.SplitMix64(5)
    circs, want = [], []
    for i in range(24):
        n = rng.between(6, 18)
        fault = rng.between(1, 50) if i % 3 == 0 else None
        g = miters.layered_cone_miter(2000 + i, n, rng.between(100, 1200), fault_seed=fault)
        circs.append(es.fastlec_es_load_aig(g.to_aig()))
        want.append(oracle.check(g.to_aag(), threads=8))
    res = es.fastlec_es_check_batch(circs)
    got = [r["cex"] if r["verdict"] else None for r in res]
    assert got == want
    # any permutation of the batch gives the same per-circuit answers
    perm = list(range(len(circs)))[::-1]
    res2 = es.fastlec_es_check_batch([circs[i] for i in perm])
    assert [r["cex"] if r["verdict"] else None for r in res2] == [want[i] for i in perm]


def test_batch_null_entry_reports_its_own_status():
    """A null handle inside a batch: that entry's verdict is FASTLEC_ERR_INVALID, the other
    entries carry the oracle's answers, and the call reports the first bad entry."""
    import ctypes
    gs = [miters.layered_cone_miter(2100 + i, 12, 600, fault_seed=(7 if i == 2 else None)) for i in range(4)]
    circs = [es.fastlec_es_load_aig(g.to_aig()) for g in gs]
    want = [oracle.check(g.to_aag(), threads=8) for g in gs]
    handles = [circs[0].handle.value, None, circs[1].handle.value, circs[2].handle.value, None,
               circs[3].handle.value]
    arr = (ctypes.c_void_p * len(handles))(*handles)
    res = (es.fastlec_es_result * len(handles))()
    rc = es.lib().fastlec_es_check_batch(arr, len(handles), None, res)
    assert rc == es.FASTLEC_ERR_INVALID
    assert b"entry 1" in es.lib().fastlec_es_last_error()
    assert res[1].verdict == es.FASTLEC_ERR_INVALID and res[4].verdict == es.FASTLEC_ERR_INVALID
    assert res[1].patterns_evaluated == 0 and res[4].patterns_evaluated == 0
    got = [res[j].cex if res[j].verdict else None for j in (0, 2, 3, 5)]
    assert got == want
    assert want[2] is not None


def test_invalid_ranges_rejected():
    c = es.fastlec_es_load_aig(miters.minterm_miter(10, [3]).to_aag())
    with pytest.raises(es.EsError) as ei:
        es.fastlec_es_check(c, begin_word=5, end_word=5)
    assert ei.value.code == es.FASTLEC_ERR_INVALID
    with pytest.raises(es.EsError):
        es.fastlec_es_check(c, begin_word=0, end_word=1 << 10)


@pytest.mark.parametrize("kernel", ["specialized", "interp"])
def test_full_space_coverage_n32(kernel):
    """Single-minterm circuits over 32 inputs: the kernel must reach every part of 2^32."""
    rng = miters.SplitMix64(32)
    targets = [0, (1 << 32) - 1, (1 << 31) - 1, 1 << 31] + [rng.below(1 << 32) for _ in range(8)]
    for t in targets:
        c = es.fastlec_es_load_aig(miters.minterm_miter(32, [t]).to_aig())
        assert gpu_answer(c, kernel=kernel) == t


def test_full_size_mac8_fault():
    name = "mac8_fused_separate_f2"
    c = es.fastlec_es_load_aig(miters.workload(name).to_aig())
    for kernel in ("specialized", "interp"):
        assert gpu_answer(c, kernel=kernel) == expected(name)


@pytest.mark.parametrize("name", ["mult16_array_booth", "mac8_fused_separate"])
def test_full_size_equivalent(name):
    """Equivalent at 2^32: verdict from both kernels; the oracle agrees on sampled patterns, and
    on the whole space where its exhaustive run is recorded in the goldens."""
    g = miters.workload(name)
    c = es.fastlec_es_load_aig(g.to_aig())
    for kernel in ("specialized", "interp"):
        r = es.fastlec_es_check(c, kernel=kernel)
        assert r["verdict"] == es.FASTLEC_EQUIVALENT and r["patterns_evaluated"] == 1 << 32
    rng = miters.SplitMix64(len(name))
    ps = np.array([rng.next_u64() >> 32 for _ in range(1 << 14)], dtype=np.uint64)
    assert not oracle.Circuit(g.to_aag()).miter(ps).any()
    golden = json.load(open(os.path.join(GOLDEN, "expected.json")))
    if name in golden:
        assert golden[name]["lowest_failure"] is None


def test_batch_graph_replays_match_eager():
    """check_batch records a hipGraph on first use and replays it: every replay, with eager
    launches in between, must give the eager per-circuit answers."""
    rng = miters.SplitMix64(21)
    gs = []
    for i in range(20):
        n = rng.between(8, 17)
        gs.append(miters.layered_cone_miter(3000 + i, n, rng.between(150, 1500),
                                            fault_seed=(rng.between(1, 60) if i % 4 == 0 else None)))
    circs = [es.fastlec_es_load_aig(g.to_aig()) for g in gs]
    eager = [gpu_answer(c, kernel="interp") for c in circs]
    assert eager == [oracle.check(g.to_aag(), threads=8) for g in gs]
    for rep in range(4):
        res = es.fastlec_es_check_batch(circs)
        assert [r["cex"] if r["verdict"] else None for r in res] == eager
        assert gpu_answer(circs[rep], kernel="interp") == eager[rep]
        assert gpu_answer(circs[-1 - rep], kernel="specialized") == eager[-1 - rep]
    for K in (1, 4):
        res = es.fastlec_es_check_batch(circs, words_per_thread=K, wg_size=128)
        assert [r["cex"] if r["verdict"] else None for r in res] == eager
    res = es.fastlec_es_check_batch(circs, kernel="interp_hbm")
    assert [r["cex"] if r["verdict"] else None for r in res] == eager


def test_cached_schedule_refits_larger_batch(monkeypatch):
    """A tuned schedule is cached per (rows, cones, work) bucket.  When a later batch in the same
    bucket has larger value files, the cached workgroup may not fit in LDS any more; the cached
    choice must be re-fitted (or re-tuned), never launched as is.  The hook forces the choice
    K=4, B=8, 128 threads, which fits about 80 rows."""
    monkeypatch.setenv("FASTLEC_ES_TUNE_FORCE", "4,8,128")
    rng = miters.SplitMix64(78)
    picked = []
    for i in range(80):
        size = rng.between(1100, 2000)
        g = miters.layered_cone_miter(7000 + i, 10, size, fault_seed=(i if i % 3 == 0 else None))
        c = es.fastlec_es_load_aig(g.to_aig())
        info = c.info()
        if 2048 <= info["num_ands_tfi"] < 4096:
            picked.append((10 + info["peak_live_slots"] + 2, g, c))
    picked.sort(key=lambda t: t[0])
    assert picked[0][0] <= 70 and picked[-1][0] >= 84
    for rows, g, c in picked:
        print("batch of one cone, rows", rows, flush=True)
        res = es.fastlec_es_check_batch([c])
        assert (res[0]["cex"] if res[0]["verdict"] else None) == oracle.check(g.to_aag(), threads=8), rows


@pytest.mark.parametrize("n", [40, 52, 63])
def test_high_input_bits_in_word_ranges(n):
    """Inputs above bit 36 of the pattern index come from the high word of the base index.
    Minterm miters whose failing patterns have high bits set are checked on word windows
    around the targets: a window holding a target reports it (the lower one first), a window
    just below it is equivalent with exactly its patterns simulated."""
    rng = miters.SplitMix64(n)
    hi = rng.below(1 << (n - 1)) | (1 << (n - 1))      # top input set
    lo = hi - 64 * rng.between(3, 200) - rng.below(64)  # a second target a few words lower
    g = miters.minterm_miter(n, [hi, lo])
    c = es.fastlec_es_load_aig(g.to_aig())
    for kernel in KERNELS:
        w_lo, w_hi = lo // 64, hi // 64
        r = es.fastlec_es_check(c, kernel=kernel, begin_word=w_lo - 5, end_word=w_hi + 7)
        assert r["verdict"] == es.FASTLEC_NONEQUIVALENT and r["cex"] == lo, (kernel, r)
        r = es.fastlec_es_check(c, kernel=kernel, begin_word=w_lo + 1, end_word=w_hi + 1)
        assert r["verdict"] == es.FASTLEC_NONEQUIVALENT and r["cex"] == hi, (kernel, r)
        r = es.fastlec_es_check(c, kernel=kernel, begin_word=w_hi - 300, end_word=w_hi)
        if w_lo < w_hi - 300:
            assert r["verdict"] == es.FASTLEC_EQUIVALENT and r["patterns_evaluated"] == 64 * 300, (kernel, r)
    # the oracle agrees on the same windows (it scans patterns directly)
    o = oracle.Circuit(g.to_aag())
    assert o.lowest_failure(64 * (lo // 64 - 5), 64 * (hi // 64 + 7), threads=4)[0] == lo


def test_specialized_lds_spills_match_oracle(monkeypatch):
    """The asm block capped at 24 VGPRs keeps most values in LDS spill slots (ds_write_b32 /
    ds_read_b32); answers on the stored workloads and on layered cones must not change."""
    monkeypatch.setenv("FASTLEC_ES_JIT_VGPR_CAP", "24")
    for name in ("mult12_array_booth_f1", "mult12_array_booth_f3", "mac8_fused_separate_f1", "mult16_array_booth_f2"):
        c = es.fastlec_es_load_aig(miters.workload(name).to_aig())
        src = es.fastlec_es_specialized_source(c, 3)
        assert "LDS spill operations" in src, name
        print("spilled kernel", name, flush=True)
        assert gpu_answer(c, kernel="specialized") == expected(name), name
    rng = miters.SplitMix64(88)
    for i in range(4):
        g = miters.layered_cone_miter(8800 + i, rng.between(12, 18), rng.between(800, 3000),
                                      fault_seed=(i + 1 if i % 2 else None))
        c = es.fastlec_es_load_aig(g.to_aig())
        assert gpu_answer(c, kernel="specialized") == oracle.check(g.to_aag(), threads=8), i


def test_per_gate_fallback_emitter_matches_oracle(monkeypatch):
    """The last-resort emitter (one asm statement per gate, compiler register allocation), used
    when a cone is too wide even for LDS spill slots, forced here on stored workloads."""
    monkeypatch.setenv("FASTLEC_ES_JIT_EMIT", "0")
    for name in ("mult6_array_wallace_f1", "mult12_array_booth_f2", "mac8_fused_separate_f2"):
        c = es.fastlec_es_load_aig(miters.workload(name).to_aig())
        assert "one asm block" not in es.fastlec_es_specialized_source(c, 3)
        assert gpu_answer(c, kernel="specialized") == expected(name), name
