"""The host layer of the library (argument validation, the work planner, the
tile cost model, error reporting) under AddressSanitizer and
UndefinedBehaviorSanitizer: api.cpp is rebuilt with both on its host code,
linked with the kernels' objects, and the host-only tests (test_abi,
test_planner, test_tile_model: no device call) run against that build in a
child process with the ASan runtime preloaded.  Any sanitizer report ends the
child with a non-zero status (UBSan does not recover)."""
import os
import shutil
import subprocess
import sys

import pytest

from paper_2506_03477_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_TESTS = ["tests/test_abi.py", "tests/test_planner.py", "tests/test_tile_model.py"]


@pytest.mark.timeout(900)
@pytest.mark.skipif(not os.path.exists(B.HIPCC) and shutil.which("hipcc") is None,
                    reason="hipcc is not installed")
def test_host_layer_under_asan_ubsan():
    lib = B.build_host_sanitized()
    rt = B.asan_runtime()
    assert os.path.exists(rt), rt
    env = dict(os.environ)
    env["LD_PRELOAD"] = rt + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    env["CHI0_LIB"] = lib
    # the interpreter's own allocations are never freed at exit: leak checks off
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-s", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu"] + HOST_TESTS,
                       cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True, timeout=840)
    out = r.stdout
    reports = [l for l in out.splitlines()
               if "runtime error:" in l or "ERROR: AddressSanitizer" in l]
    assert r.returncode == 0 and not reports, "\n".join(reports) or out[-4000:]
    assert " passed" in out, out[-2000:]
