"""Host-side checks of the C library that need no GPU.

* the library loads and exports every function include/fastlec_es.h declares;
* AIGER loading, validation and error codes;
* the planner's instruction streams, replayed on the host with the kernels'
  bundle semantics, agree with the oracle pattern by pattern (this pins the
  reference-count slot map independently of any kernel);
* the specialized kernel source compiles for gfx950 through hipRTC.
"""
import json
import os
import re

import numpy as np
import pytest

import miters
import oracle
import paper_2512_06627_amd as es

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "fastlec_es.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fastlec_es_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_function():
    names = header_functions()
    assert len(names) >= 16
    lib = es.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(s[0] for s in es.SIGNATURES) == names


def test_load_errors_and_info():
    with pytest.raises(es.EsError) as ei:
        es.fastlec_es_load_aig(b"aag 3 1 1 1 1\n2\n4 6\n6\n6 2 4\n")
    assert ei.value.code == es.FASTLEC_ERR_UNSUPPORTED
    with pytest.raises(es.EsError) as ei:
        es.fastlec_es_load_aig(b"hello")
    assert ei.value.code == es.FASTLEC_ERR_PARSE
    with pytest.raises(es.EsError) as ei:
        es.fastlec_es_load_aig(miters.minterm_miter(64, [1]).to_aig())
    assert ei.value.code == es.FASTLEC_ERR_UNSUPPORTED
    g = miters.workload("mult16_array_booth")
    a = es.fastlec_es_load_aig(g.to_aag()).info()
    b = es.fastlec_es_load_aig(g.to_aig()).info()
    assert a == b
    assert a["num_pis"] == 32 and a["num_ands_tfi"] == len(g.tfi_ands())
    assert 50 <= a["peak_live_slots"] <= 200


def test_hand_fixture_errors_match_oracle_reader(golden_dir):
    spec = json.load(open(os.path.join(golden_dir, "hand_worked.json")))
    for name, s in spec.items():
        if name.startswith("_"):
            continue
        data = open(os.path.join(golden_dir, "hand", name), "rb").read()
        if "error" in s:
            with pytest.raises(es.EsError) as ei:
                es.fastlec_es_load_aig(data)
            assert ei.value.code == {"parse": -1, "unsupported": -2}[s["error"]], name
        else:
            es.fastlec_es_load_aig(data)


def _replay_vs_oracle(g, bundle, halfwords):
    c = es.fastlec_es_load_aig(g.to_aig())
    o = oracle.Circuit(g.to_aag())
    n = g.num_inputs
    for hw in halfwords:
        word = es.fastlec_es_host_replay(c, bundle, hw, 1)[0]
        ps = np.array([32 * hw + j for j in range(32)], dtype=np.uint64)
        if n < 5:
            ps = ps % np.uint64(1 << n)
        bits = o.miter(ps)
        assert word == int(sum(int(b) << j for j, b in enumerate(bits))), (hw, bundle)


@pytest.mark.parametrize("bundle", [0, 1, 4, 8, 16])
def test_plan_replay_matches_oracle(bundle):
    # bundle 0: the register tier's encoded stream, read the way that kernel reads it
    rng = miters.SplitMix64(bundle)
    for name in ("mult6_array_wallace_f1", "mult12_array_booth_f3", "mac8_fused_separate_f1"):
        g = miters.workload(name)
        H = 1 << (g.num_inputs - 5)
        _replay_vs_oracle(g, bundle, [0, H - 1] + [rng.below(H) for _ in range(6)])
    for i in range(6):
        g = miters.layered_cone_miter(300 + i, 14, 800, fault_seed=i + 1)
        _replay_vs_oracle(g, bundle, [rng.below(1 << 9) for _ in range(4)])
    for n, t in ((3, [5]), (5, [31]), (9, [300])):
        g = miters.minterm_miter(n, t)
        _replay_vs_oracle(g, bundle, range(max(1, 1 << (n - 5)) if n >= 5 else 1))


def _lut_replay_vs_oracle(g, halfwords):
    c = es.fastlec_es_load_aig(g.to_aig())
    o = oracle.Circuit(g.to_aag())
    n = g.num_inputs
    for hw in halfwords:
        word = es.fastlec_es_host_replay_specialized(c, hw, 1)[0]
        ps = np.array([32 * hw + j for j in range(32)], dtype=np.uint64)
        if n < 5:
            ps = ps % np.uint64(1 << n)
        assert word == int(sum(int(b) << j for j, b in enumerate(o.miter(ps)))), hw


def test_specialized_lut_program_matches_oracle(golden_dir):
    """The specialized kernel's program (LUT mapping, scalar steps, plan-time words), run on the host."""
    rng = miters.SplitMix64(9)
    for name in ("mult6_array_wallace_f1", "mult12_array_booth_f2", "mult16_array_booth", "mac8_fused_separate_f2"):
        g = miters.workload(name)
        H = 1 << (g.num_inputs - 5)
        _lut_replay_vs_oracle(g, [0, H - 1] + [rng.below(H) for _ in range(12)])
    for i in range(10):
        n = rng.between(6, 14)
        g = miters.layered_cone_miter(700 + i, n, rng.between(200, 1500), fault_seed=(i if i % 2 else None))
        H = max(1, 1 << (n - 5))
        _lut_replay_vs_oracle(g, sorted({0, H - 1, rng.below(H), rng.below(H)}))
    for n, t in ((1, [1]), (3, [5]), (5, [31]), (9, [300]), (13, [8000, 77])):
        _lut_replay_vs_oracle(miters.minterm_miter(n, t), range(max(1, 1 << max(0, n - 5))))
    spec = json.load(open(os.path.join(golden_dir, "hand_worked.json")))
    for name, s in spec.items():
        if name.startswith("_") or "error" in s:
            continue
        c = es.fastlec_es_load_aig(open(os.path.join(golden_dir, "hand", name), "rb").read())
        w = es.fastlec_es_host_replay_specialized(c, 0, 1)[0]
        assert ((w & -w).bit_length() - 1 if w else None) == s["expect"], name


def test_specialized_kernel_compiles_for_gfx950():
    c = es.fastlec_es_load_aig(miters.workload("mult6_array_wallace").to_aig())
    info = es.fastlec_es_compile_specialized(c, 2)
    assert info["code_bytes"] > 1000
    src = es.fastlec_es_specialized_source(c, 2)
    assert "fes_es_kernel" in src and "v_bitop3_b32" in src


def test_classes_match_oracle_on_host():
    """fastlec_es_classes runs on the host: first row of each hash value, as the oracle."""
    from oracle import rsim
    r = np.random.default_rng(4)
    for rows in (0, 1, 7, 5000):
        h = r.integers(0, 40, size=rows, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15)
        assert np.array_equal(es.fastlec_es_classes(h), rsim.classes(h))


def test_simulation_argument_errors_without_gpu():
    from miters.miter import mult_circuit
    c = es.fastlec_es_load_aig(mult_circuit("array", 3).to_aig())
    for call in (lambda: es.fastlec_es_simulate(c, 1, 0, 1),          # no words
                 lambda: es.fastlec_es_simulate(c, None, 4, 1),       # inputs needed
                 lambda: es.fastlec_es_signature_hash(0, 1, 1, 1, 1),  # null signature
                 lambda: es.fastlec_es_signature_hash(1, 0, 1, 1, 1)):  # no rows
        with pytest.raises(es.EsError) as ei:
            call()
        assert ei.value.code == -5


def test_runtime_model_properties():
    """fastlec_es_predict (host only): the paper's form, linear in gates and exponential in
    inputs beyond the fixed costs; the compile estimate does not depend on the range."""
    g = miters.layered_cone_miter(44, 30, 3000)
    c = es.fastlec_es_load_aig(g.to_aig())
    full = es.fastlec_es_predict(c)
    half = es.fastlec_es_predict(c, 0, 1 << (30 - 7))   # half the 2^24 64-bit words
    assert all(v > 0 for v in full.values())
    assert full["interp_ms"] > full["specialized_ms"]
    assert 1.9 < full["interp_ms"] / half["interp_ms"] <= 2.0
    assert 1.9 < full["specialized_ms"] / half["specialized_ms"] <= 2.0
    assert full["compile_ms"] == half["compile_ms"] > 100
    small = es.fastlec_es_load_aig(miters.layered_cone_miter(44, 30, 1000).to_aig())
    assert es.fastlec_es_predict(small)["interp_ms"] < full["interp_ms"]
    with pytest.raises(es.EsError):
        es.fastlec_es_predict(c, 5, 3)


def test_batch_of_null_entries_reports_each_entry():
    """Every entry null: no device is needed; each entry's verdict is FASTLEC_ERR_INVALID and the
    call returns that status, naming the first entry."""
    import ctypes
    arr = (ctypes.c_void_p * 3)(None, None, None)
    res = (es.fastlec_es_result * 3)()
    for r in res:
        r.verdict = 99
    assert es.lib().fastlec_es_check_batch(arr, 3, None, res) == es.FASTLEC_ERR_INVALID
    assert all(r.verdict == es.FASTLEC_ERR_INVALID for r in res)
    assert b"entry 0" in es.lib().fastlec_es_last_error()
    assert es.lib().fastlec_es_check_batch(None, 3, None, res) == es.FASTLEC_ERR_INVALID


def test_specialized_kernels_compile_together():
    """Several circuits' kernels compiled in one call: each kernel reachable afterwards (a
    single compile of each circuit then costs nothing and reports its code object), and one
    call with a repeated circuit compiles it once.  How the kernels are split into programs
    (one program, or one per compile helper process) is pinned in test_rtc_helper_cpu.py."""
    cs = [es.fastlec_es_load_aig(miters.layered_cone_miter(800 + i, 25, 1200).to_aig()) for i in range(6)]
    assert es.fastlec_es_compile_specialized_many(cs + cs[:2], 3) > 0
    for c in cs:
        r = es.fastlec_es_compile_specialized(c, 3)
        assert r["compile_ms"] == 0
        assert r["code_bytes"] > 0
    assert es.fastlec_es_compile_specialized_many(cs, 3) == 0
    with pytest.raises(es.EsError):
        es.fastlec_es_compile_specialized_many(cs, 0)


# ---- three-AND XORs fused into one interpreter instruction ----------------------------------

def _xor_roots(g):
    """Gates k = ~t1 & ~t2 with t1 = x & y, t2 = ~x & ~y, t1 and t2 read only by k, taken in
    variable order; a gate already taken as such a root is not the inner gate of another.
    Counted over the output cone (gates some output depends on)."""
    n = g.num_inputs
    cone, stack = set(), [o >> 1 for o in g.outputs]
    while stack:
        v = stack.pop()
        if v > n and v not in cone:
            cone.add(v)
            stack.extend(r >> 1 for r in g.ands[v - n - 1])
    readers = {}
    for r0, r1 in g.ands:
        for r in (r0, r1):
            readers[r >> 1] = readers.get(r >> 1, 0) + 1
    for o in g.outputs:
        readers[o >> 1] = readers.get(o >> 1, 0) + 1
    roots = set()
    for k, (l1, l2) in enumerate(g.ands):
        if not (l1 & 1 and l2 & 1):
            continue
        t1, t2 = l1 >> 1, l2 >> 1
        if t1 == t2 or t1 <= n or t2 <= n or readers[t1] != 1 or readers[t2] != 1:
            continue
        if (t1 - n - 1) in roots or (t2 - n - 1) in roots:
            continue
        x, y = g.ands[t1 - n - 1]
        p, q = g.ands[t2 - n - 1]
        if {p, q} == {x ^ 1, y ^ 1} and x >> 1 != y >> 1:
            roots.add(k)
    return sum(1 for k in roots if n + 1 + k in cone)


def _parity(n, form):
    from miters.aig import Aig
    g = Aig(n)
    acc = g.input(0)
    for i in range(1, n):
        acc = getattr(g, form)(acc, g.input(i))
    g.add_output(acc)
    return g


@pytest.mark.parametrize("form", ["XOR", "XOR_alt", "XOR_andor"])
def test_xor_fusion_parity_chains(form):
    """Each of the three common three-AND XOR forms is fused; the bundled streams (which run the
    fused copy) replay to the oracle's miter words on every pattern."""
    g = _parity(9, form)
    c = es.fastlec_es_load_aig(g.to_aig())
    assert c.info()["num_xors"] == 8 == _xor_roots(g)
    for bundle in (1, 4, 8, 16):
        _replay_vs_oracle(g, bundle, range(1 << 4))


def test_xor_fusion_skips_shared_inner_gates():
    """A half adder's carry reads x & y too, so its XOR keeps its three ANDs."""
    from miters.aig import Aig
    g = Aig(6)
    s = g.XOR(g.input(0), g.input(1))
    carry = g.AND(g.input(0), g.input(1))
    g.add_output(g.AND(s, g.input(2)))
    g.add_output(g.AND(carry, g.input(3)))
    g.add_output(g.XOR(g.input(4), g.input(5)))   # this one is fused
    c = es.fastlec_es_load_aig(g.to_aig())
    assert c.info()["num_xors"] == 1 == _xor_roots(g)
    for bundle in (1, 4, 16):
        _replay_vs_oracle(g, bundle, range(2))


@pytest.mark.parametrize("name", ["mult12_array_booth", "mac8_fused_separate", "mult16_array_booth"])
def test_xor_fusion_count_matches_definition(name):
    g = miters.workload(name)
    c = es.fastlec_es_load_aig(g.to_aig())
    assert c.info()["num_xors"] == _xor_roots(g) > 0


def test_register_stream_replay_on_wide_files_and_limits():
    # Value files near each register-tier size (104, 144, 232 rows) replay like the oracle; a
    # file above 232 rows is refused.
    rng = miters.SplitMix64(77)
    seen = set()
    for seed, n, gates in ((41, 16, 1200), (43, 18, 7000), (44, 20, 8000), (46, 16, 20000)):
        g = miters.layered_cone_miter(seed, n, gates, fault_seed=seed)
        rows = es.fastlec_es_load_aig(g.to_aig()).info()["interp_rows"]
        if rows > 232:
            with pytest.raises(es.EsError) as ei:
                es.fastlec_es_host_replay(es.fastlec_es_load_aig(g.to_aig()), 0, 0, 1)
            assert ei.value.code == es.FASTLEC_ERR_INVALID
            seen.add("over")
            continue
        seen.add(104 if rows <= 104 else 144 if rows <= 144 else 232)
        _replay_vs_oracle(g, 0, [rng.below(1 << (n - 5)) for _ in range(4)])
    g = miters.workload("mult16_array_booth_f1")
    _replay_vs_oracle(g, 0, [0, (1 << 27) - 1, rng.below(1 << 27)])
    assert seen == {104, 144, 232, "over"}, seen
