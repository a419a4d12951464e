"""The oracle (C) and the library's host-side planning code (C++, no HIP)
built for the CPU with AddressSanitizer and UndefinedBehaviorSanitizer and
run on small cases (tests/sanitize/*): any out-of-bounds access, leak, use
after free, signed overflow or misaligned access fails the test.  CPU only;
skipped where the compiler has no sanitizer runtime."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _build(tmp_path, compiler, sources, out, extra):
    exe = str(tmp_path / out)
    cmd = [compiler] + SAN + extra + ["-o", exe] + sources
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        if "asan" in r.stdout.lower() or "sanitizer" in r.stdout.lower():
            pytest.skip("no sanitizer runtime: " + r.stdout[-300:])
        raise AssertionError("build failed:\n" + r.stdout)
    return exe


def _run(exe):
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       env=ENV, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout[-4000:]


def test_oracle_under_sanitizers(tmp_path):
    exe = _build(tmp_path, "gcc", [os.path.join(HERE, "sanitize", "oracle_check.c")],
                 "oracle_check", ["-std=c11", "-Wno-unknown-pragmas", "-lm"])
    _run(exe)


def test_host_plan_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1904_02108_amd", "csrc")
    exe = _build(tmp_path, "g++", [os.path.join(HERE, "sanitize", "plan_check.cpp"),
                                   os.path.join(csrc, "host_plan.cpp")],
                 "plan_check", ["-std=c++17", "-I" + os.path.join(ROOT, "include"), "-I" + csrc])
    _run(exe)
