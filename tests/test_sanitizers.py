"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
the library's host-only paths (gate table, fusion, planning, pass schedules,
cache-blocked grouping, tuning, argument checks) through a C++ driver linked
against a sanitized copy of libcast, and the C oracle through a C driver."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")


def _load(name, path):
    import importlib.util
    spec = importlib.util.spec_from_file_location(name, path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _run(exe):
    r = subprocess.run([exe], env=ENV, capture_output=True, text=True, timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


@pytest.mark.slow
def test_library_host_code_sanitized():
    b = _load("_cast_build_asan", os.path.join(ROOT, "paper_2503_19894_amd", "build.py"))
    _run(b.build_sanitized(os.path.join(ROOT, "tests", "native", "host_driver.cpp")))


def test_oracle_sanitized():
    b = _load("_oracle_build_asan", os.path.join(ROOT, "oracle", "build.py"))
    _run(b.build_sanitized(os.path.join(ROOT, "tests", "native", "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "_build_asan")))
