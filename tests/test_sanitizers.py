"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the oracle (driven over every entry point and its edge shapes by
tests/helpers/oracle_driver.c), the serving scheduler's host logic
(tests/helpers/sched_test.cpp) and the binary64 device math built for the host
(tests/helpers/math_test.cpp). Any report aborts the program
(-fno-sanitize-recover), so a clean exit with the expected output is the pass.
GPU code is never built with a sanitizer: on the hipcc line the flag applies
to the host pass only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HELPERS = os.path.join(ROOT, "tests", "helpers")
CSRC = os.path.join(ROOT, "paper_2010_09341_amd", "csrc")
SAN = "-fsanitize=address,undefined"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(exe, stdin=None):
    res = subprocess.run([exe], input=stdin, capture_output=True, text=True, env=ENV,
                         timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr
    return res.stdout


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", SAN, "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-ffp-contract=off", "-Wall",
                    os.path.join(ROOT, "oracle", "vegas_oracle.c"),
                    os.path.join(HELPERS, "oracle_driver.c"), "-lm", "-o", exe], check=True)
    assert _run(exe).strip() == "ok"


def test_scheduler_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sched_test")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", SAN, "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-Wall", "-I" + CSRC,
                    os.path.join(HELPERS, "sched_test.cpp"), "-o", exe], check=True)
    assert _run(exe).strip() == "ok"


def test_device_math_host_build_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc is not installed")
    exe = str(tmp_path / "math_test")
    subprocess.run([hipcc, "-O1", "-g", "-Xarch_host", SAN, "-Xarch_host",
                    "-fno-sanitize-recover=all", "-I" + CSRC,
                    os.path.join(HELPERS, "math_test.cpp"), "-o", exe],
                   check=True, capture_output=True)
    xs = ["e 0.5", "e -745.2", "e 709.7", "l 1e-310", "l 3.5", "p 0.25 1.5", "p 1e-300 64"]
    out = _run(exe, "\n".join(xs) + "\n").split()
    assert len(out) == len(xs)
