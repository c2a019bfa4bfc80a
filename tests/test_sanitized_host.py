"""The C ABI's host code (argument checks, workspace carving, work-table
packing, graph set-up, the deformation-graph and incidence builders) under
AddressSanitizer and UndefinedBehaviorSanitizer: the library's CPU tests run
in a child process against the host-sanitized build, which aborts on the first
report.  CPU only; skipped when the product build's objects are absent."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2104_00359_amd")


@pytest.mark.slow
def test_library_cpu_tests_pass_under_asan_and_ubsan():
    sys.path.insert(0, PKG)
    try:
        import build_sanitized
    finally:
        sys.path.remove(PKG)
    if not os.path.isdir(build_sanitized.build.BUILD):
        pytest.skip("no product build objects (run build() first)")
    try:
        lib = build_sanitized.build_sanitized()
    except FileNotFoundError as e:
        pytest.skip(str(e))
    env = dict(os.environ, SHV_LIBRARY=lib, LD_PRELOAD=build_sanitized.runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_lib_cpu.py")], cwd=ROOT, env=env,
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=900)
    print(r.stdout[-3000:])
    assert r.returncode == 0
    assert "ERROR: AddressSanitizer" not in r.stdout and "runtime error:" not in r.stdout
