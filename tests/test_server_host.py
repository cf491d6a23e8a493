"""The serving runtime on the host, without a GPU: server.cpp and the
library's host helpers built with the host compiler against a stand-in for the
HIP runtime (tests/cpp/fake_hip, tests/cpp/fake_device.cpp), driven by
tests/cpp/server_test.cpp through the C ABI with camera, polling, scheduler
and completion threads, once under the thread sanitizer and once under the
address and undefined-behaviour sanitizers (leaks included).  The driver
checks every published image against the window definition, alone and in a
three-stream mix, the hold / staging back-pressure / admission / gap policies
and that concurrent whole-cycle submits share launches."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = [os.path.join(ROOT, "paper_1511_03390_amd", "csrc", "server.cpp"),
           os.path.join(ROOT, "paper_1511_03390_amd", "csrc", "capi.cpp"),
           os.path.join(ROOT, "tests", "cpp", "fake_device.cpp"),
           os.path.join(ROOT, "tests", "cpp", "server_test.cpp")]
FLAGS = ["-std=c++17", "-O1", "-g", "-Wno-attributes", "-I", os.path.join(ROOT, "tests", "cpp", "fake_hip"),
         "-I", os.path.join(ROOT, "paper_1511_03390_amd", "csrc")]


def build_and_run(tmp_path, name, sanitize, env):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / name)
    r = subprocess.run([cxx, *FLAGS, *sanitize, *SOURCES, "-o", exe, "-lpthread"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600, env={**os.environ, **env})
    out = run.stdout + run.stderr
    assert run.returncode == 0, out[-6000:]
    assert "all checks passed" in run.stdout
    assert "WARNING: ThreadSanitizer" not in out and "ERROR: AddressSanitizer" not in out
    assert "runtime error" not in out
    return run.stdout


def test_server_threads_under_thread_sanitizer(tmp_path):
    out = build_and_run(tmp_path, "server_tsan", ["-fsanitize=thread"],
                        {"TSAN_OPTIONS": "halt_on_error=1 exitcode=66"})
    print(out)


def test_server_under_address_and_undefined_sanitizers(tmp_path):
    build_and_run(tmp_path, "server_asan", ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
                  {"ASAN_OPTIONS": "detect_leaks=1", "UBSAN_OPTIONS": "halt_on_error=1"})
