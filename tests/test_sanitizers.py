"""The oracle and the library's host-side plan construction under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only): each program exercises its entry points on small
valid and malformed inputs and must finish without a sanitizer report (any report, including
a leak in the oracle, ends it with a nonzero status)."""
import os
import subprocess

import pytest


def _run(exe, leaks):
    env = dict(os.environ, ASAN_OPTIONS=f"detect_leaks={1 if leaks else 0}:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    return r.returncode, r.stdout + r.stderr


def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    from tests.native import build_sanitized
    rc, out = _run(build_sanitized.oracle_sanitized(), leaks=True)
    assert rc == 0, out[-3000:]
    assert "oracle sanitize ok" in out


def test_plan_construction_under_address_and_undefined_behaviour_sanitizers():
    from tests.native import build_sanitized
    exe = build_sanitized.plan_sanitized()
    if exe is None:
        pytest.skip("hipcc not available")
    # the HIP runtime's own allocations outlive main: leak checking is off for this one
    rc, out = _run(exe, leaks=False)
    assert rc == 0, out[-3000:]
    assert "plan sanitize ok" in out
