"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc) and driven through every entry point on small and degenerate shapes
by tests/oracle_sanitize.c: no out-of-bounds access, use after free, leak
or undefined arithmetic, and every call returns its success code."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "sip_oracle.c")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           os.path.join(HERE, "oracle_sanitize.c"), SRC, "-o", exe, "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    p = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "shapes ok" in p.stdout
