"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a
program that calls every oracle entry point (oracle/sanitize_check.c) on
small lattices, extents 1 and 2 included, both couplings and both
order-parameter schemes, one and four threads.  Any sanitizer report aborts
the program."""
from __future__ import annotations

import subprocess

import pytest


def test_oracle_is_clean_under_asan_and_ubsan():
    from oracle import build
    try:
        exe = build.build_sanitize_check()
    except (OSError, subprocess.CalledProcessError) as e:  # no gcc sanitizer runtime
        pytest.skip(f"sanitizer build unavailable: {e}")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env={"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0",
                            "UBSAN_OPTIONS": "print_stacktrace=1", "PATH": "/usr/bin:/bin"})
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitize check ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
