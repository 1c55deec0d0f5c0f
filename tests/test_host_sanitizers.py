"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
libpsp's C ABI host logic through tests/host/abi_driver.c, and the oracle's
C FFT through tests/host/oracle_fft_driver.c.  A sanitizer report, a leak or
a wrong return code fails the test."""
import os
import subprocess

import pytest

from tests.host import sanitized

ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out and "LeakSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


def test_abi_host_logic_under_sanitizers():
    out = _run(sanitized.build_abi_driver())
    assert "0 failures" in out


def test_oracle_fft_under_sanitizers():
    out = _run(sanitized.build_oracle_driver())
    assert "0 failures" in out
