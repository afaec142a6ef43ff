"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

tests/host/sanitize_setup.cpp drives the host setup (strength, RS first pass, classical interpolation,
Galerkin products, aggressive coarsening, ILU(0) and ILUT, smoother data, level schedules), the factor
diagnostics and the input validation on small matrices; it is compiled here with g++ together with
setup_host.cpp and diagnostics.cpp, sanitizers on, and must exit cleanly with no report.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2112_14681_amd", "csrc")


@pytest.mark.parametrize("sanitizer", ["address,undefined"])
def test_host_setup_under_sanitizers(tmp_path, sanitizer):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "sanitize_setup")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           f"-fsanitize={sanitizer}", "-fno-sanitize-recover=all", "-I", "/opt/rocm/include",
           os.path.join(ROOT, "tests", "host", "sanitize_setup.cpp"), os.path.join(CSRC, "setup_host.cpp"),
           os.path.join(CSRC, "diagnostics.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "failures: 0" in r.stdout
