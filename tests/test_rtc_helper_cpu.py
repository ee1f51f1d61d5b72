"""The compile helper program (paper_2512_06627_amd/rtc/fastlec_es_rtc.cpp): grouped hipRTC
compiles run in child processes side by side, since hipRTC serializes compiles inside one process.
hipRTC needs no GPU, so this runs on the CPU: the helper produces the same code object as the
library's in-process compile, reports a failing source with a non-zero status and hipRTC's log,
a grouped compile of 24 kernels is split into one program per helper (one program in this process
when helpers are turned off), fewer than 4 kernels stay one program, programs whose helper fails
or hangs past its time limit are compiled in this process, and helpers inherit none of the host
program's files.  comgr's on-disk compile cache is turned off in the child
processes, so every compile is a real one."""
import os
import shutil
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


def _grouped_compile(k, procs, seed, lib_path=None, env_extra=None, marker=None):
    code = ("import sys, os; sys.path.insert(0, %r)\n"
            "import miters, paper_2512_06627_amd as es\n"
            "if %r: es.LIB_PATH = %r\n"
            "if %r: fd = os.open(%r, os.O_RDONLY); os.set_inheritable(fd, True)\n"
            "cs = [es.fastlec_es_load_aig(miters.layered_cone_miter(%d + i, 18, 900).to_aig()) for i in range(%d)]\n"
            "es.fastlec_es_compile_specialized_many(cs, 3)\n"
            "print('compiled', all(es.fastlec_es_compile_specialized(c, 3)['compile_ms'] == 0 for c in cs))\n"
            % (ROOT, bool(lib_path), lib_path, bool(marker), marker, seed, k))
    env = dict(os.environ, FASTLEC_ES_RTC_PROCS=procs, FASTLEC_ES_TRACE="1", AMD_COMGR_CACHE="0", **(env_extra or {}))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "compiled True" in r.stdout, r.stdout  # every kernel cached after the grouped compile
    return r.stderr


@pytest.mark.parametrize("k,procs,programs", [(24, "4", 4), (24, "0", 1), (3, "4", 1)])
def test_grouped_compile_in_helper_processes(k, procs, programs):
    err = _grouped_compile(k, procs, 7400)
    assert f"compiling {k} kernels as {programs} programs" in err, err[-3000:]


def _library_with_helper(tmp_path, script):
    """A copy of the library beside a stand-in helper (a shell script)."""
    shutil.copy(es.LIB_PATH, tmp_path / os.path.basename(es.LIB_PATH))
    helper = tmp_path / "fastlec_es_rtc"
    helper.write_text("#!/bin/sh\n" + script)
    helper.chmod(0o755)
    return str(tmp_path / os.path.basename(es.LIB_PATH))


def test_failing_helper_falls_back_to_in_process_compile(tmp_path):
    # Every helper fails: every program is then compiled in the process, and every kernel is
    # still there.  The stand-in also lists its open files: the inheritable file the host program
    # opened is not among them (children keep only stdin, stdout and stderr).
    marker = tmp_path / "marker_file"
    marker.write_text("x")
    lib = _library_with_helper(tmp_path, 'ls -l /proc/$$/fd > "$FES_TEST_FDS.$$" 2>&1\nexit 3\n')
    err = _grouped_compile(6, "3", 7500, lib, env_extra={"FES_TEST_FDS": str(tmp_path / "fds")}, marker=str(marker))
    assert "compiling 6 kernels as 3 programs" in err, err[-3000:]
    assert err.count("helper failed on program") == 3, err[-3000:]
    reports = [f for f in os.listdir(tmp_path) if f.startswith("fds.")]
    assert len(reports) == 3
    for f in reports:
        text = (tmp_path / f).read_text()
        assert "marker_file" not in text, text


def test_hung_helper_is_killed_at_its_deadline(tmp_path):
    # Helpers that never finish: each is killed after the time limit and its program compiled in
    # the process.
    lib = _library_with_helper(tmp_path, "exec sleep 120\n")
    err = _grouped_compile(4, "2", 7600, lib, env_extra={"FASTLEC_ES_RTC_TIMEOUT_S": "1"})
    assert "compiling 4 kernels as 2 programs" in err, err[-3000:]
    assert err.count("timed out; killing it") == 2, err[-3000:]
    assert err.count("helper failed on program") == 2, err[-3000:]
