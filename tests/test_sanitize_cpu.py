"""The host-side planner path built with AddressSanitizer and UndefinedBehaviorSanitizer.

tests/sanitize/host_driver.cpp runs the AIGER reader, the slot planner (bundles 1, 4, 8, 16, each
validated by symbolic replay), the LUT mapper (scalar-unit and all-VALU policies), the block
emitter (all option combinations), the simulation plan and the sub-miter extraction of every
candidate pair on every file, and prints the LUT program's miter words at chosen half-words and
a hash of the sub-miters; those must equal the oracles'.  Host code only: nothing here runs on a GPU.
"""
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

import miters
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2512_06627_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not os.path.exists(CLANG):
        pytest.skip("clang++ not found")
    out = str(tmp_path_factory.mktemp("san") / "host_driver")
    srcs = [os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp")] + [
        os.path.join(CSRC, f) for f in ("aig.cpp", "plan.cpp", "lut.cpp", "emit_block.cpp", "sweep.cpp")]
    cmd = [CLANG, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROOT, "include"),
           "-I/opt/rocm/include", "-I" + CSRC] + srcs + ["-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return out


def _circuits(golden_dir):
    out = []
    for name in ("mult6_array_wallace_f1", "mult12_array_booth_f2", "mac8_fused_separate_f1", "mult16_array_booth"):
        out.append((name, miters.workload(name)))
    rng = miters.SplitMix64(55)
    for i in range(8):
        n = rng.between(6, 18)
        out.append((f"layered{i}", miters.layered_cone_miter(5500 + i, n, rng.between(100, 1500),
                                                             fault_seed=(i + 3 if i % 2 else None))))
    for n, t in ((0, []), (1, [1]), (4, [3, 9 % 16]), (6, [63]), (12, [64, 4000])):
        out.append((f"minterm{n}", miters.minterm_miter(n, t)))
    return out


def test_planner_path_under_sanitizers(driver, tmp_path, golden_dir):
    circs = _circuits(golden_dir)
    files = []
    for k, (name, g) in enumerate(circs):
        p = tmp_path / f"c{k}.aig"
        p.write_bytes(g.to_aig())
        files.append(str(p))
    spec = json.load(open(os.path.join(golden_dir, "hand_worked.json")))
    hand = [n for n in sorted(spec) if not n.startswith("_")]
    for n in hand:
        files.append(os.path.join(golden_dir, "hand", n))
    hws = [0, 1, 37, 1000, 123456789]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver, ",".join(map(str, hws))] + files, capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    out = r.stdout.strip().splitlines()
    sweeps = [l for l in out if " sweep " in l]
    lines = [l for l in out if " sweep " not in l]
    assert len(lines) == len(files)
    # sub-miters of every target, from the same classes, equal the virtual-sweeping oracle's
    from oracle import rsim, sweep
    by_index = {int(l.split()[0]): l.split()[2:] for l in sweeps}
    for k, (name, g) in enumerate(circs):
        aag = g.to_aag()
        n = g.num_inputs
        words = np.array([[((i + 1) * 0x9E3779B1 + w * 0x85EBCA77) % (1 << 32) for w in range(4)] for i in range(n)],
                         dtype=np.uint32).reshape(n, 4)
        sig = rsim.simulate(aag, words)
        cls = rsim.classes(rsim.signature_hash(sig)[0]).tolist()
        pol = (sig[:, 0] & 1).astype(int).tolist()
        h, count = 0xcbf29ce484222325, 0
        for t in sweep.targets(cls, n):
            for ch in sweep.submiter_aag(aag, cls, pol, t)[0]:
                h = ((h ^ ch) * 0x100000001B3) % (1 << 64)
            count += 1
        assert by_index[k] == [str(count), str(h)], name
    for line, (name, g) in zip(lines, circs):
        fields = line.split()
        o = oracle.Circuit(g.to_aag())
        n = g.num_inputs
        for hw, got in zip(hws, fields[1:]):
            h = hw % (1 << (n - 5)) if n >= 5 else 0
            ps = np.array([32 * h + j for j in range(32)], dtype=np.uint64)
            if n < 5:
                ps = ps % np.uint64(max(1, 1 << n))
            want = sum(int(b) << j for j, b in enumerate(o.miter(ps)))
            assert int(got) == want, (name, hw)
    for line, n in zip(lines[len(circs):], hand):
        if "error" in spec[n]:
            assert " error " in line, (n, line)
