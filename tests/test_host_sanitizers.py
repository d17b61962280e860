"""Host setup code under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/native/host_sanitize.cpp drives the library's host-side numerics (the
factor products of App. B, the single-branch preconditioner of Sec. IV-D,
the plant step and the closed-loop KPIs of Sec. V-B) on random systems and
their error paths.  It is built here with the host sources, the sanitizers
on the host pass only (no GPU code is built or run), and must print "ok"
with no sanitizer report.  The oracle is NumPy and has no native code to
sanitize."""

import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1604_01074_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_host_setup_code_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "host_sanitize"
    sanitizers = []
    for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"):
        sanitizers += ["-Xarch_host", flag]
    cmd = [HIPCC, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *sanitizers,
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(HERE, "native", "host_sanitize.cpp"), os.path.join(CSRC, "smpc_setup.cpp"),
           os.path.join(CSRC, "smpc_loop.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr
