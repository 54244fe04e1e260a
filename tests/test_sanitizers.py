"""The library's host code under AddressSanitizer + UndefinedBehaviorSanitizer
and under ThreadSanitizer (CPU only, no device work).

tests/sanitize/host_driver.cpp drives the planner, the INT8 block bound, the
footprint, the entry points' argument checks and a dry-run server fed by four
submitting threads (plus a server whose launches fail on the host); it is
linked against sanitizer builds of the host sources (tests/sanitize/build.py)
and must finish with no finding and no failed expectation.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _build(kind):
    sys.path.insert(0, os.path.join(ROOT, "tests", "sanitize"))
    try:
        import build as sanitize_build
    finally:
        sys.path.pop(0)
    if not os.path.exists(os.path.join(ROOT, "_build", "mmp")):
        pytest.skip("the product objects are not built")
    return sanitize_build.build(kind)


@pytest.mark.parametrize("kind", ["asan", "tsan"])
def test_host_code_under_sanitizer(kind):
    exe = _build(kind)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["TSAN_OPTIONS"] = "halt_on_error=1:second_deadlock_stack=1"
    env["HIP_VISIBLE_DEVICES"] = ""  # host paths only, never a device
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "host driver: 0 failures" in out
    for word in ("ERROR: AddressSanitizer", "runtime error:", "WARNING: ThreadSanitizer", "LeakSanitizer"):
        assert word not in out, out[-4000:]
