"""Algorithm 1's driver (csrc/driver.h, host code) on a mock of the device side: the hook
after the pilot (the learned run trains there and replaces the coarsest level's pilot walks)
runs once, after the pilot's first measurement; the levels are measured again before any
sample size is computed; and the hook that does nothing leaves the driver as it was."""
import subprocess

import pytest

from tests.native import build_native


def test_driver_after_pilot_hook():
    exe = build_native.driver_hook()
    if exe is None:
        pytest.skip("g++ not available")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "driver hook ok" in r.stdout
