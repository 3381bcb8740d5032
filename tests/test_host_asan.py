"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU).

The host-sanitized debug build (paper_2607_06834_amd/build_asan.py,
build_host_asan: host pass instrumented, device code as in the product
library) is loaded, with the shared ASan runtime preloaded, in a pytest
process of its own that runs the tests calling the host-only entry points:
descriptor validation and planning (ptafs_estimate, the standardized form's
plan), the timing-model projection and the per-pulsar Gram quantities
(ptafs_std_precompute, ptafs_std_precompute_cw) against the oracle, and the
error paths of invalid descriptors.  Any sanitizer report fails the test.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_TESTS = ["tests/test_std_host.py", "tests/test_abi.py"]


def _stale(lib, build):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    srcs = [os.path.join(build.CSRC, f) for f in os.listdir(build.CSRC)]
    srcs += [os.path.join(build.INCLUDE, f) for f in os.listdir(build.INCLUDE)]
    srcs += [os.path.abspath(build.__file__), os.path.join(os.path.dirname(build.__file__), "build.py")]
    return any(os.path.getmtime(s) > t for s in srcs)


@pytest.mark.slow
def test_host_code_under_sanitizers():
    from paper_2607_06834_amd import build_asan as build
    lib = build.ASAN_LIB
    if _stale(lib, build):
        build.build_host_asan()
    rt = build.asan_runtime()
    env = dict(os.environ)
    pre = env.get("LD_PRELOAD", "")
    env["LD_PRELOAD"] = rt + (" " + pre if pre else "")      # the runtime must come first
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:detect_odr_violation=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["PTAFS_TEST_LIB"] = lib
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider", *HOST_TESTS]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "AddressSanitizer" not in out, out[-6000:]
    assert "runtime error:" not in out, out[-6000:]
    summary = [ln for ln in r.stdout.splitlines() if ln.strip()][-1]
    assert " passed" in summary and "skipped" not in summary, summary
