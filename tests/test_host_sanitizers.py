"""The C ABI's argument checks and error paths under AddressSanitizer, LeakSanitizer and
UndefinedBehaviorSanitizer (host code only): tests/abi_sanitized.c linked against a build of
the library whose host sources carry the sanitizers. No device is needed for this leg; the GPU
leg (small solves on every path) is tests/test_gpu_host_sanitizers.py."""
import os
import subprocess

from paper_2512_12515_amd import build as B

ENV = dict(os.environ,
           ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def test_argument_checks_clean_under_sanitizers():
    try:
        exe = B.build_sanitized()
    except RuntimeError as e:
        if "run build() first" not in str(e):
            raise
        B.build()
        exe = B.build_sanitized()
    r = subprocess.run([exe], env=ENV, capture_output=True, text=True, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ALL OK" in r.stdout, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
