"""The runtime model's decisions on the host (no GPU): the server's specialized-tier rule and
the batch's longest-processing-time cost, on a fixed job set, against the model the library
publishes through fastlec_es_predict.

The server compiles a job's specialized kernel when its remaining interpreter time at its share
of the device (the jobs on the interpreter share each step equally) exceeds the predicted
specialized time of that work plus twice the predicted compile time.  The model driver (tests/sanitize/model_driver.cpp, built with
AddressSanitizer and UBSan) calls the library's decision function directly.  The batch's price
of a grouped compile in helper processes is checked against compile times measured on MI355X's
host.
"""
import os
import re
import subprocess

import pytest

import miters
import paper_2512_06627_amd as es

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2512_06627_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not os.path.exists(CLANG):
        pytest.skip("clang++ not found")
    out = str(tmp_path_factory.mktemp("model") / "model_driver")
    cmd = [CLANG, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I" + CSRC, os.path.join(ROOT, "tests", "sanitize", "model_driver.cpp"), os.path.join(CSRC, "model.cpp"),
           "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return out


def _jobs():
    out = [("mult6", miters.workload("mult6_array_wallace")), ("mult12", miters.workload("mult12_array_booth")),
           ("mult16", miters.workload("mult16_array_booth")), ("mac8", miters.workload("mac8_fused_separate"))]
    for i, (n, size) in enumerate(((18, 600), (24, 3000), (28, 5000), (34, 20000))):
        out.append((f"layered{n}", miters.layered_cone_miter(700 + i, n, size)))
    return out


def _lut_steps(c):
    return int(re.search(r"(\d+) LUT steps", es.fastlec_es_specialized_source(c, 3)).group(1))


def test_server_tier_rule_follows_the_model(driver):
    rows, expect = [], []
    for name, g in _jobs():
        c = es.fastlec_es_load_aig(g.to_aig())
        i = c.info()
        n = i["num_pis"]
        gates = i["num_instrs"] - 2 * i["num_xors"]
        luts = _lut_steps(c)
        words = 1 << max(0, n - 6)
        for left in (words, max(1, words // 16)):  # whole space left, a sixteenth left
            p = es.fastlec_es_predict(c, words - left, words)
            for sharing in (1, 8, 64):
                rows.append(f"{gates} {i['interp_rows']} {luts} {32.0 * 2 * left if n >= 6 else 2.0 ** n} {sharing}")
                expect.append((name, left, sharing, p))
    r = subprocess.run([driver], input="\n".join(rows) + "\n", capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = r.stdout.split("\n")
    wanted = {}
    for line, (name, left, sharing, p) in zip(lines, expect):
        want, rem, comp, alone, lpt, spec = line.split()
        rem, comp, alone, lpt, spec = float(rem), float(comp), float(alone), float(lpt), float(spec)
        assert alone == pytest.approx(p["interp_ms"], rel=1e-6), name
        assert comp == pytest.approx(p["compile_ms"], rel=1e-6), name
        assert spec == pytest.approx(p["specialized_ms"], rel=1e-6), name
        assert rem == pytest.approx(sharing * p["interp_ms"], rel=1e-6), name
        assert lpt == pytest.approx(p["interp_ms"], rel=1e-6), name  # LPT orders by the model's time
        assert int(want) == (sharing * p["interp_ms"] > p["specialized_ms"] + 2.0 * p["compile_ms"]), (name, sharing)
        wanted[(name, left, sharing)] = int(want)
    # the fixed set spans both sides of the rule: a 2^34-pattern cone is worth a compile even
    # alone, the 6x6 miter never is, and the 16x16 miter becomes worth one only when it shares
    # the device (at the register tier's rate it takes about 0.13 s alone, against 0.13 s of
    # compile counted twice)
    assert wanted[("layered34", 1 << 28, 1)] == 1
    assert all(wanted[("mult6", 64, s)] == 0 for s in (1, 8, 64))
    assert wanted[("mult16", 1 << 26, 1)] == 0 and wanted[("mult16", 1 << 26, 8)] == 1


# Grouped compiles measured on the GPU machine's host (16 cores, comgr's compile cache off): k kernels
# of layered cones (n = 24, about N AND gates; generator seeds 700 onward, in this order) split
# into p programs compiled side by side by compile helper processes; wall seconds.
GROUP_COMPILES = [((600, 2), {1: 0.155, 2: 0.141}), ((600, 4), {1: 0.183, 2: 0.156, 4: 0.152}),
                  ((600, 16), {1: 0.344, 2: 0.241, 4: 0.185, 8: 0.174}), ((2000, 2), {1: 0.158, 2: 0.146}),
                  ((2000, 4), {1: 0.192, 2: 0.163, 4: 0.139}),
                  ((2000, 16), {1: 0.390, 2: 0.260, 4: 0.200, 8: 0.163}),
                  ((15000, 8), {1: 0.450, 2: 0.303, 4: 0.210, 8: 0.171})]


def test_group_compile_model_against_measured_compiles(driver):
    """The batch's price of a grouped compile (fixed cost with a helper's start-up, then each
    kernel's part over the helpers) against the measured wall times: never more than 5% low (a low
    price would route cones whose compile does not pay) and at most 20% high."""
    rows, want = [], []
    seed = 700
    for (gates, k), by_programs in GROUP_COMPILES:
        luts = []
        for _ in range(k):
            c = es.fastlec_es_load_aig(miters.layered_cone_miter(seed, 24, gates).to_aig())
            seed += 1
            luts.append(_lut_steps(c))
        for p, seconds in by_programs.items():
            rows.append(f"{p} {k} " + " ".join(map(str, luts)))
            want.append(((gates, k, p), 1000.0 * seconds))
    r = subprocess.run([driver, "group"], input="\n".join(rows) + "\n", capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-3000:]
    got = [float(x) for x in r.stdout.split()]
    assert len(got) == len(want)
    for pred, (case, ms) in zip(got, want):
        assert 0.95 * ms <= pred <= 1.20 * ms, (case, pred, ms)
