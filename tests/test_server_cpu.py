"""The server's request scheduler (paper_1303_4538_amd/csrc/sip_sched.cpp)
on the CPU: the same scheduler the library runs, over a CPU backend that
solves every request with the oracle (tests/server_cpu/fake_backend.cpp),
driven through the C ABI by tests/server_cpu/server_driver.cpp.  The
scenarios cover admission under the budget, least-recently-used eviction,
the protection of systems named by queued requests, the queue limit,
argument errors, factorisation, allocation and step failures, cancellation
at shutdown, and concurrent submit / poll / release / stats from many
threads; every solved request must equal its own oracle solve bitwise.

The driver is built twice: with ThreadSanitizer (ROCm's clang, whose
runtime intercepts every condition-variable wait the C++ library uses) and
with AddressSanitizer + UndefinedBehaviorSanitizer (gcc).  Any report fails
the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1303_4538_amd", "csrc")
SOURCES = [os.path.join(CSRC, "sip_sched.cpp"), os.path.join(CSRC, "sip_host.cpp"),
           os.path.join(HERE, "server_cpu", "fake_backend.cpp"), os.path.join(HERE, "server_cpu", "server_driver.cpp")]
ORACLE = os.path.join(ROOT, "oracle", "sip_oracle.c")
SCENARIOS = 12

ROCM_CLANG = "/opt/rocm/llvm/bin/clang"


def build(tmp_path, cc, cxx, san):
    obj = str(tmp_path / "oracle.o")
    exe = str(tmp_path / "server_driver")
    subprocess.check_call([cc, "-O1", "-g", "-std=c99", "-ffp-contract=off", *san, "-c", ORACLE, "-o", obj])
    subprocess.check_call([cxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread", *san,
                           "-I" + os.path.join(ROOT, "include"), *SOURCES, obj, "-o", exe])
    return exe


def run(exe, env):
    p = subprocess.run([exe], capture_output=True, text=True, env=dict(os.environ, **env), timeout=600)
    out = p.stdout + p.stderr
    assert p.returncode == 0, out[-6000:]
    assert f"{SCENARIOS} scenarios passed" in p.stdout, out[-6000:]
    assert "Sanitizer" not in out, out[-6000:]


@pytest.mark.skipif(not os.path.exists(ROCM_CLANG + "++"), reason="needs ROCm's clang (ThreadSanitizer runtime)")
def test_scheduler_under_thread_sanitizer(tmp_path):
    exe = build(tmp_path, ROCM_CLANG, ROCM_CLANG + "++", ["-fsanitize=thread"])
    run(exe, {"TSAN_OPTIONS": "halt_on_error=1 exitcode=66 second_deadlock_stack=1"})


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs gcc")
def test_scheduler_under_address_sanitizer(tmp_path):
    exe = build(tmp_path, "gcc", "g++", ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"])
    run(exe, {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0:exitcode=23",
              "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1:exitcode=24"})
