"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The host sources (setup of the reference element, mesh, PML classification and layout, the C ABI, the PML
schemes, batching and the adjoint driver) are built instrumented (``build.py --sanitize``; device code is not
instrumented) and the CPU library tests run against that build in a child process with the sanitizer runtime
preloaded: any heap overflow, use after free or undefined behaviour in the host paths aborts the child.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2006_02551_amd import build  # noqa: E402


def _stale():
    if not os.path.exists(build.SAN_LIB):
        return True
    t = os.path.getmtime(build.SAN_LIB)
    srcs = [os.path.join(build.CSRC, f) for f in os.listdir(build.CSRC)]
    srcs.append(os.path.join(ROOT, "include", "wdg.h"))
    return any(os.path.getmtime(s) > t for s in srcs)


@pytest.fixture(scope="module")
def san_env():
    try:
        build.hipcc()
        build.sanitizer_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    if _stale():
        build.build_sanitized()
    return build.sanitizer_env()


def test_sanitized_build_is_instrumented(san_env):
    out = subprocess.run(["nm", "-D", build.SAN_LIB], capture_output=True, text=True).stdout
    assert "__asan_report_load8" in out and "__ubsan_handle" in out


def test_library_cpu_suite_under_sanitizers(san_env):
    code = ("import sys; sys.path.insert(0, %r); import pytest; from paper_2006_02551_amd import wdg; "
            "assert wdg.LIB_PATH == %r, wdg.LIB_PATH; "
            "sys.exit(pytest.main(['-x', '-q', '-p', 'no:cacheprovider', %r]))"
            % (ROOT, build.SAN_LIB, os.path.join(ROOT, "tests", "test_library_cpu.py")))
    r = subprocess.run([sys.executable, "-c", code], env=san_env, capture_output=True, text=True, cwd=ROOT)
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
    assert "passed" in r.stdout and "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
