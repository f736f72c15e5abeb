"""Host-side checks of the C ABI (run without a GPU): the library loads, it
exports every function include/pentbatch.h declares, the binding's signature
table matches the header, and argument errors are reported before any HIP
call is made."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1807_07382_amd import pentbatch as pb

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "pentbatch.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pent_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_core_entry_points():
    names = declared_functions()
    for n in ("pent_factor", "pent_solve", "pent_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = pb.lib()
    for name in declared_functions():
        assert hasattr(L, name), f"{name} declared but not exported"


def test_binding_covers_header():
    assert sorted(pb.SIGNATURES) == declared_functions()


def test_factor_rejects_bad_arguments_without_hip():
    L = pb.lib()
    a = np.zeros(4)
    p = a.ctypes.data
    assert not L.pent_factor(0, p, p, p, p, p)
    assert L.pent_last_status() == pb.INVALID_VALUE
    assert not L.pent_factor(-5, p, p, p, p, p)
    assert L.pent_last_status() == pb.INVALID_VALUE
    assert not L.pent_factor(4, None, p, p, p, p)
    assert L.pent_last_status() == pb.INVALID_VALUE
    assert not L.pent_factor(4, p, p, p, p, None)
    assert L.pent_last_status() == pb.INVALID_VALUE
    assert not L.pent_factor(2 ** 31, p, p, p, p, p)
    assert L.pent_last_status() == pb.INVALID_VALUE
    assert not L.pent_factor_d4(0, 1.0)
    assert L.pent_last_status() == pb.INVALID_VALUE
    assert not L.pent_factor_d4(8, float("nan"))
    assert L.pent_last_status() == pb.INVALID_VALUE
    assert not L.pent_factor_d4(8, float("inf"))
    assert L.pent_last_status() == pb.INVALID_VALUE


def test_null_handle_is_rejected_everywhere():
    L = pb.lib()
    buf = (ctypes.c_double * 8)()
    assert L.pent_solve(None, buf, 1, 1, None) == pb.INVALID_VALUE
    assert L.pent_solve_strided(None, buf, 1, 1, None) == pb.INVALID_VALUE
    assert L.pent_solve_noalloc(None, buf, 1, 1, None) == pb.INVALID_VALUE
    assert L.pent_get_factors(None, buf, buf, buf, buf) == pb.INVALID_VALUE
    assert L.pent_get_diagonals(None, buf, buf, buf, buf, buf) == pb.INVALID_VALUE
    assert L.pent_size(None) == -1
    assert L.pent_set_schedule(None, 0, 0) == pb.INVALID_VALUE


def test_forged_handle_is_rejected():
    """A pointer that is not a live handle fails the handle check (magic word)."""
    L = pb.lib()
    junk = (ctypes.c_uint64 * 64)()
    h = ctypes.cast(junk, ctypes.c_void_p)
    assert L.pent_solve(h, None, 0, 0, None) == pb.INVALID_VALUE
    assert L.pent_solve_noalloc(h, None, 0, 0, None) == pb.INVALID_VALUE
    assert L.pent_destroy(h) == pb.INVALID_VALUE
    assert L.pent_size(h) == -1


def test_destroy_null_is_noop():
    assert pb.lib().pent_destroy(None) == pb.OK
    assert pb.lib().pent_last_status() == pb.OK


@pytest.mark.parametrize("st", range(0, 10))
def test_status_strings(st):
    s = pb.lib().pent_status_string(st)
    assert isinstance(s, bytes) and len(s) > 0
    if st == 9:
        assert s == b"unknown status"
    else:
        assert s != b"unknown status"


def test_python_errors_on_bad_shapes():
    with pytest.raises(ValueError):
        pb.Plan.factor(np.zeros(3), np.zeros(3), np.zeros(4), np.zeros(3), np.zeros(3))


def test_cyclic_rejects_bad_arguments_without_hip():
    L = pb.lib()
    a = np.zeros(8)
    p = a.ctypes.data
    assert not L.pent_cyclic_factor(4, p, p, p, p, p)
    assert L.pent_last_status() == pb.INVALID_VALUE
    assert not L.pent_cyclic_factor(8, p, None, p, p, p)
    assert L.pent_last_status() == pb.INVALID_VALUE
    assert not L.pent_cyclic_factor_d4(4, 1.0)
    assert L.pent_last_status() == pb.INVALID_VALUE
    assert not L.pent_cyclic_factor_d4(8, float("nan"))
    assert L.pent_last_status() == pb.INVALID_VALUE
    buf = (ctypes.c_double * 8)()
    assert L.pent_cyclic_solve(None, buf, 1, 1, None) == pb.INVALID_VALUE
    assert L.pent_cyclic_cn_rhs(None, buf, 1, buf, 1, 1, None) == pb.INVALID_VALUE
    assert L.pent_cyclic_bordering(None, buf, buf) == pb.INVALID_VALUE
    assert L.pent_cyclic_destroy(None) == pb.OK
    assert L.pent_cyclic_cn_step(None, buf, 1, buf, 1, 1, None) == pb.INVALID_VALUE
    assert L.pent_cyclic_set_schedule(None, 0, 32) == pb.INVALID_VALUE
    assert L.pent_cyclic_check(None) == pb.INVALID_VALUE
    assert L.pent_check(None) == pb.INVALID_VALUE
    junk = (ctypes.c_uint64 * 64)()
    h = ctypes.cast(junk, ctypes.c_void_p)
    assert L.pent_cyclic_solve(h, buf, 1, 1, None) == pb.INVALID_VALUE
    assert L.pent_cyclic_destroy(h) == pb.INVALID_VALUE


def test_rewrite_rejects_bad_arguments_without_hip():
    L = pb.lib()
    buf = (ctypes.c_double * 64)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    need = L.pent_rewrite_workspace_size(8, 4)
    assert need == 256 + 16 * 8 * 4
    assert L.pent_rewrite_workspace_size(0, 4) == 0
    assert L.pent_solve_rewrite(0, p, p, p, p, p, 4, p, 4, 4, p, need, None) == pb.INVALID_VALUE
    assert L.pent_solve_rewrite(8, p, p, p, p, p, 3, p, 4, 4, p, need, None) == pb.INVALID_VALUE
    assert L.pent_solve_rewrite(8, p, p, p, p, p, 4, p, 4, 3, p, need, None) == pb.INVALID_VALUE
    assert L.pent_solve_rewrite(8, None, p, p, p, p, 4, p, 4, 4, p, need, None) == pb.INVALID_VALUE
    assert L.pent_solve_rewrite(8, p, p, p, p, p, 4, p, 4, 4, p, need - 1, None) == pb.SIZE_MISMATCH
    assert L.pent_solve_rewrite(8, p, p, p, p, p, 4, p, 0, 4, p, need, None) == pb.OK
    assert L.pent_rewrite_check(None, 8, None, None) == pb.INVALID_VALUE


def test_stream_copy_rejects_bad_arguments_without_hip():
    L = pb.lib()
    buf = (ctypes.c_double * 64)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    # shapes other than the five measured ones, bad sizes, null pointers
    for ta, wd in ((1, 1), (3, 1), (4, 2), (1, 8), (0, 4), (2, 4)):
        assert L.pent_stream_copy_shaped(p, 8, p, 8, 8, 8, ta, wd, None) == pb.INVALID_VALUE
    assert L.pent_stream_copy_shaped(p, 8, p, 8, 0, 8, 1, 2, None) == pb.INVALID_VALUE
    assert L.pent_stream_copy_shaped(p, 4, p, 8, 8, 8, 1, 2, None) == pb.INVALID_VALUE
    assert L.pent_stream_copy_shaped(None, 8, p, 8, 8, 8, 2, 2, None) == pb.INVALID_VALUE
    assert L.pent_stream_copy_shaped(p, 8, p, 8, 8, 0, 4, 1, None) == pb.OK  # empty batch: no-op
    assert L.pent_stream_copy(p, 8, None, 8, 8, 8, None) == pb.INVALID_VALUE
