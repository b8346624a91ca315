"""The host plan builder under AddressSanitizer and UndefinedBehaviorSanitizer:
the planner's parity and error-path tests (tests/test_plan_parity.py) run in a
child process against a build of the library whose plan.cpp is instrumented,
and must pass with no sanitizer report."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_plan_parity_under_asan_and_ubsan(tmp_path):
    from paper_1601_06984_amd import build as B
    if not all(os.path.exists(os.path.join(B.BUILD, s + ".o")) for s in B.HIP_SOURCES):
        pytest.skip("the library's objects are not built")
    lib = B.build_sanitized_host(str(tmp_path))
    env = B.sanitizer_env(lib, str(tmp_path))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_plan_parity.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    reports = glob.glob(str(tmp_path / "asan*")) + glob.glob(str(tmp_path / "ubsan*"))
    text = "".join(open(f).read() for f in reports)
    assert not reports, text[:4000]
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert " passed" in r.stdout
