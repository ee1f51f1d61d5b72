"""The server's host threads under ThreadSanitizer, on the CPU.

tests/sanitize/server_race_driver.cpp runs submitter, poller and stats threads against a server's
step loop and compile thread, and destroys a second server with work in flight; every answer
must equal the circuit checked alone.  It is built with the thread sanitizer together with the
library's host sources and tests/sanitize/fake_device.cpp, a host stand-in for the GPU that runs
the interpreter and specialized-kernel launches on the CPU from the same descriptors and streams
(the HIP runtime finds no device in a process built with the thread sanitizer).  Two runs: slices
sized for many small steps with the compile tier by estimate, and every job sent to the compile
thread.  Any sanitizer report fails the test.
"""
import concurrent.futures
import os
import re
import subprocess

import pytest

import miters

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2512_06627_amd", "csrc")
SAN = os.path.join(ROOT, "tests", "sanitize")
CLANG = "/opt/rocm/llvm/bin/clang++"
HOST_SOURCES = ("aig", "capi", "emit_block", "lut", "model", "plan", "runtime", "server", "sweep")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not os.path.exists(CLANG):
        pytest.skip("clang++ not found")
    d = tmp_path_factory.mktemp("race")
    flags = ["-std=c++17", "-O1", "-g", "-fsanitize=thread", "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__",
             "-I" + os.path.join(ROOT, "include"), "-I/opt/rocm/include", "-I" + CSRC]
    srcs = [os.path.join(CSRC, f + ".cpp") for f in HOST_SOURCES] + [
        os.path.join(SAN, "fake_device.cpp"), os.path.join(SAN, "server_race_driver.cpp")]

    def compile_one(src):
        obj = str(d / (os.path.basename(src) + ".o"))
        r = subprocess.run([CLANG] + flags + ["-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    out = str(d / "server_race")
    r = subprocess.run([CLANG, "-fsanitize=thread", "-o", out] + objs + ["-lpthread"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return out


@pytest.fixture(scope="module")
def circuits(tmp_path_factory):
    d = tmp_path_factory.mktemp("race_aig")
    # small cones finish in one slice; n = 18 and 20 take 8 and 32 slices of the smallest size
    specs = [(8001, 12, 400, 1), (8002, 14, 600, None), (8003, 13, 500, 2), (8004, 14, 400, None),
             (8005, 18, 300, 3), (8006, 18, 350, None), (8007, 20, 300, None), (8008, 20, 250, 4)]
    files = []
    for k, (seed, n, gates, fault) in enumerate(specs):
        p = d / f"c{k}.aig"
        p.write_bytes(miters.layered_cone_miter(seed, n, gates, fault_seed=fault).to_aig())
        files.append(str(p))
    return files


@pytest.mark.parametrize("jit", ["1", "2"])
def test_server_threads_have_no_data_races(driver, circuits, jit):
    env = dict(os.environ, FASTLEC_ES_SERVER_JIT=jit, FASTLEC_ES_SERVER_RATE="1000000000",
               FASTLEC_ES_SERVER_STEP_MS="1", FASTLEC_ES_TRACE="1", FASTLEC_ES_BATCH_JIT="2",
               TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([driver] + circuits, capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-8000:])
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-8000:]
    assert r.stdout.strip().endswith("ok 96"), r.stdout
    assert "batches from 2 threads: 0 wrong" in r.stdout, r.stdout
    # AUTO batches routed cones to their (existing) kernels: each such batch ran its compile
    # thread beside its interpreter launches
    assert "batch: routing every cone whose kernel exists" in r.stderr, r.stderr[-3000:]
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("server:")][0]
    assert " 0 mismatches, 0 errors" in line, line
    if jit == "2":
        assert " 0 specialized slices" not in line, line  # the compile thread took part
    else:
        steps = int(line.split(" specialized slices, ")[1].split()[0])
        assert steps >= 16, line  # many steps: submissions and polls overlap the loop
