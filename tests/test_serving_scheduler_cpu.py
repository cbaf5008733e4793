"""The serving scheduler of the host runtime on the CPU (no GPU).

tests/schedsim builds paper_2109_04528_amd/csrc/tor_runtime.cpp with g++ or
clang against a host-only stand-in for the HIP calls it makes (streams are
threads, events complete in stream order, "device" memory is host memory)
and stand-ins for the kernel launchers, whose per-root values make a
matrix's sum independent of its split and wrong if a root runs twice, not at
all, or on another request's slots.  The driver serves the policy and sizes
of the sanitized GPU driver, a mixed stream with arrivals over time, a
saturated burst under the default policy, chunked launches with express
launches off, a stream of both arithmetic paths, and a destroy with requests
in flight; every served value must
equal the lone evaluation's, and every scenario must finish in time.  It
runs under AddressSanitizer with UndefinedBehaviorSanitizer and under
ThreadSanitizer (clang's, which understands the condition-variable waits the
scheduler polls with), at two simulated kernel rates so that launches
overlap differently."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SIM = os.path.join(ROOT, "tests", "schedsim")
SOURCES = [os.path.join(ROOT, "paper_2109_04528_amd", "csrc", "tor_runtime.cpp"),
           os.path.join(SIM, "fakehip.cpp"), os.path.join(SIM, "stubs.cpp"), os.path.join(SIM, "driver.cpp")]
CLANG = "/opt/rocm/llvm/bin/clang++"


def build(tmp_path, compiler, flags, name):
    exe = str(tmp_path / name)
    cmd = [compiler, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags,
           "-I", os.path.join(SIM, "fake"), "-I", os.path.join(ROOT, "include"), *SOURCES, "-lpthread", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    return exe


def run(exe, rate, env_extra):
    env = dict(os.environ, SCHEDSIM_RATE=rate, **env_extra)
    res = subprocess.run([exe, "150"], capture_output=True, text=True, env=env, timeout=200)
    assert res.returncode == 0, (res.returncode, res.stdout[-2000:], res.stderr[-4000:])
    assert res.stdout.strip().splitlines()[-1] == "done 0"
    assert "WARNING: ThreadSanitizer" not in res.stderr and "runtime error" not in res.stderr, res.stderr[-4000:]


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_scheduler_under_asan_and_ubsan(tmp_path):
    exe = build(tmp_path, "g++", ["-fsanitize=address,undefined"], "schedsim_asan")
    for rate in ("2e10", "2e9"):
        run(exe, rate, {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1",
                        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})


@pytest.mark.skipif(not os.path.exists(CLANG), reason="no clang with ThreadSanitizer")
def test_scheduler_under_tsan(tmp_path):
    exe = build(tmp_path, CLANG, ["-fsanitize=thread"], "schedsim_tsan")
    for rate in ("2e10", "2e9"):
        run(exe, rate, {"TSAN_OPTIONS": "halt_on_error=1"})
