"""The bracket the walk kernel puts around the exact holding-time logarithm holds for
every one of the 2^32 words (checked exhaustively on the GPU by tests/native/log_bound.hip).
The kernel's path decisions are exact because of this bound."""
import subprocess
import sys

import pytest

from tests.native import build_native

pytestmark = pytest.mark.gpu


def test_fast_log_bracket_holds_for_all_words():
    exe = build_native.log_bound()
    assert exe is not None, "hipcc needed to build the check"
    print("log_bound: all 2^32 words", file=sys.stderr, flush=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, file=sys.stderr, flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    ratio = float(r.stdout.split()[1])
    assert ratio < 1.0
