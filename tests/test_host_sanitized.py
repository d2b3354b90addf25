"""The host side of the library (planner, C-ABI argument checks, workspace
layout, surrogate set-up) under AddressSanitizer and UndefinedBehaviorSanitizer:
the host test files run in a child process against librpot_san.so, built
(host pass instrumented, device code as usual) when missing or older than a
source.  Any sanitizer report aborts the child and fails this test."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_TESTS = ["tests/test_capi_host.py", "tests/test_surrogate_host.py"]


def _stale(lib):
    if not os.path.exists(lib):
        return True
    srcs = glob.glob(os.path.join(ROOT, "paper_2311_15429_amd", "csrc", "*")) + \
        glob.glob(os.path.join(ROOT, "include", "*.h"))
    return max(os.path.getmtime(s) for s in srcs) > os.path.getmtime(lib)


@pytest.mark.timeout(900)
def test_host_tests_under_address_and_undefined_behavior_sanitizers():
    from paper_2311_15429_amd import build as B
    if _stale(B.SAN_LIB):
        B.build(sanitize=True)
    env = B.sanitizer_env()
    cmd = [sys.executable, "-m", "pytest", *HOST_TESTS, "-q", "-x", "-p", "no:cacheprovider",
           "-m", "not gpu"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=850)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error:" not in tail, tail
    # the child really ran the instrumented library under the runtime
    probe = subprocess.run([sys.executable, "-c",
                            "import paper_2311_15429_amd as p; p.load(); "
                            "m = open('/proc/self/maps').read(); "
                            "print('asan' in m and 'librpot_san.so' in m)"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert probe.stdout.strip().endswith("True"), probe.stdout + probe.stderr
