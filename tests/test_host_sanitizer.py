"""The host code of the library (schedule builder, C ABI argument checks,
hazard checker) under AddressSanitizer and UndefinedBehaviorSanitizer: the
C-ABI tests and the schedule hazard tests run again, in a child process, against
a build whose host units are instrumented (CPU only; device code is not
instrumented and no kernel runs)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_and_schedule_under_host_sanitizers():
    from paper_1809_10585_amd import build
    rt = build.asan_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime in this toolchain")
    lib = build.build_asan()
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt, HODLR_LIB_PATH=lib, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py"), os.path.join(ROOT, "tests", "test_plan_check.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out
