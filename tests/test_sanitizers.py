"""The oracle's C code and the library's host code (argument checks, handle
checks, workspace arithmetic) run their CPU tests under AddressSanitizer and
UndefinedBehaviorSanitizer without a report (tests/sanitize.py builds the
instrumented copies)."""
import os
import shutil

import pytest

from tests import sanitize

pytestmark = pytest.mark.slow


def _report(r):
    return (r.stdout[-3000:] + "\n" + r.stderr[-3000:])


def _clean(r):
    text = r.stdout + r.stderr
    return (r.returncode == 0 and "ERROR: AddressSanitizer" not in text
            and "runtime error:" not in text)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_under_asan_and_ubsan(tmp_path):
    lib = sanitize.build_oracle(str(tmp_path))
    r = sanitize.run_tests(sanitize.ORACLE_TESTS, sanitize.gcc_asan_runtime(),
                           {"PENT_ORACLE_LIB": lib})
    assert _clean(r), _report(r)
    assert " passed" in r.stdout


@pytest.mark.skipif(not os.path.exists(sanitize.HIPCC), reason="hipcc is not installed")
def test_library_host_code_under_asan_and_ubsan(tmp_path):
    lib = sanitize.build_library(str(tmp_path))
    r = sanitize.run_tests(sanitize.LIB_TESTS, sanitize.clang_asan_runtime(),
                           {"PENTBATCH_LIB": lib})
    assert _clean(r), _report(r)
    assert " passed" in r.stdout
