"""The compile helper program (paper_2512_06627_amd/rtc/fastlec_es_rtc.cpp): grouped hipRTC
compiles run in child processes side by side, since hipRTC serializes compiles inside one process.
hipRTC needs no GPU, so this runs on the CPU: the helper produces the same code object as the
library's in-process compile, reports a failing source with a non-zero status and hipRTC's log,
and a grouped compile of 24 kernels is split into two programs compiled by helpers (one program
in this process when helpers are turned off)."""
import os
import subprocess
import sys

import pytest

import miters
import paper_2512_06627_amd as es

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HELPER = os.path.join(ROOT, "paper_2512_06627_amd", "_lib", "fastlec_es_rtc")


def test_helper_matches_in_process_compile(tmp_path):
    assert os.access(HELPER, os.X_OK), "build() makes the compile helper"
    c = es.fastlec_es_load_aig(miters.layered_cone_miter(7301, 16, 1200).to_aig())
    src = tmp_path / "k.hip"
    src.write_text(es.fastlec_es_specialized_source(c, 3))
    out = tmp_path / "k.co"
    r = subprocess.run([HELPER, str(src), str(out)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert out.stat().st_size == es.fastlec_es_compile_specialized(c, 3)["code_bytes"]


def test_helper_reports_a_failing_source(tmp_path):
    src = tmp_path / "bad.hip"
    src.write_text('extern "C" __global__ void k() { this is not code }\n')
    r = subprocess.run([HELPER, str(src), str(tmp_path / "bad.co")], capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "error" in r.stderr.lower()
    assert not (tmp_path / "bad.co").exists()


@pytest.mark.parametrize("procs,programs", [("4", 2), ("0", 1)])
def test_grouped_compile_in_helper_processes(procs, programs):
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import miters, paper_2512_06627_amd as es\n"
            "cs = [es.fastlec_es_load_aig(miters.layered_cone_miter(7400 + i, 18, 900).to_aig()) for i in range(24)]\n"
            "es.fastlec_es_compile_specialized_many(cs, 3)\n"
            "print('compiled', all(es.fastlec_es_compile_specialized(c, 3)['compile_ms'] == 0 for c in cs))\n" % ROOT)
    env = dict(os.environ, FASTLEC_ES_RTC_PROCS=procs, FASTLEC_ES_TRACE="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "compiled True" in r.stdout, r.stdout  # every kernel cached after the grouped compile
    assert f"compiling 24 kernels as {programs} programs" in r.stderr, r.stderr[-3000:]
