"""The host runtime under sanitizers (CPU): tests/sanitize/host_checks.cpp
built with the host part of every source instrumented by AddressSanitizer +
UndefinedBehaviorSanitizer, and by ThreadSanitizer. The driver fuzzes the
validation of CSR and dense couplings with malformed structures, builds host
schedules, relabels random instances by reverse Cuthill-McKee and checks the
relabelled copy, and walks the argument paths of the C ABI and of the serving
interface; a sanitizer report or a failed check fails the test. (With a GPU
the same driver also runs a multi-threaded serving stream.)"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _build(kind):
    import importlib.util
    spec = importlib.util.spec_from_file_location("sbqa_build", os.path.join(ROOT, "paper_2604_01050_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.build_sanitized(kind)


SUPP = os.path.join(ROOT, "tests", "sanitize", "lsan.supp")
ENV = {
    "asan": {"ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
             "LSAN_OPTIONS": "suppressions=" + SUPP,
             "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"},
    "tsan": {"TSAN_OPTIONS": "halt_on_error=1"},
}


@pytest.mark.slow
@pytest.mark.parametrize("kind", ["asan", "tsan"])
def test_host_runtime_under_sanitizers(kind):
    exe = _build(kind)
    env = dict(os.environ, **ENV[kind])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "host checks passed" in r.stdout
    assert "Sanitizer" not in out and "runtime error" not in out, out[-4000:]
