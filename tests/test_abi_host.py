"""Host-side checks of the C ABI (no GPU needed, no kernel launched).

* the library loads and exports every function include/qft.h declares;
* argument validation returns the documented status before any HIP call;
* the host constant generator (qft_secant_table) against mpmath at 60 digits.
"""
import ctypes
import os
import re

import mpmath
import numpy as np
import pytest

import paper_1301_0763_amd as qft
from paper_1301_0763_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qft.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qft_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("qft_plan_create", "qft_plan_create_uneven", "qft_exec_fwd", "qft_exec_bwd",
              "qft_plan_destroy", "qft_plan_info", "qft_secant_table", "qft_status_string",
              "qft_last_hip_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for n in declared_functions():
        assert hasattr(L, n), n
    # the Python binding exposes the same names
    for n in declared_functions():
        assert hasattr(qft, n), n


def test_status_strings():
    for s in range(0, 9):
        assert qft.qft_status_string(s)
    assert "static scratch" in qft.qft_status_string(_lib.QFT_ERROR_SCRATCH)
    assert "size" in qft.qft_status_string(_lib.QFT_ERROR_INVALID_SIZE)


def _create(log2n, batch, dtype=0, device=0, null_plan=False):
    L = _lib.lib()
    h = ctypes.c_void_p(12345)
    st = L.qft_plan_create(None if null_plan else ctypes.byref(h), log2n, batch, dtype, device)
    return st, h.value


@pytest.mark.parametrize("log2n,status", [(0, 2), (-3, 2), (25, 2), (40, 2)])
def test_plan_create_rejects_sizes(log2n, status):
    st, h = _create(log2n, 1)
    assert st == status and h is None


@pytest.mark.parametrize("batch", [0, -1])
def test_plan_create_rejects_batch(batch):
    st, h = _create(10, batch)
    assert st == _lib.QFT_ERROR_INVALID_VALUE and h is None


def test_plan_create_rejects_dtype_and_null():
    assert _create(10, 4, dtype=7)[0] == _lib.QFT_ERROR_INVALID_VALUE
    assert _create(10, 4, null_plan=True)[0] == _lib.QFT_ERROR_INVALID_VALUE


def test_uneven_rejects():
    L = _lib.lib()
    h = ctypes.c_void_p()
    arr = (ctypes.c_int32 * 3)(5, 0, 7)
    assert L.qft_plan_create_uneven(ctypes.byref(h), arr, 3, 0, 0) == _lib.QFT_ERROR_INVALID_SIZE
    arr = (ctypes.c_int32 * 2)(5, 25)
    assert L.qft_plan_create_uneven(ctypes.byref(h), arr, 2, 0, 0) == _lib.QFT_ERROR_INVALID_SIZE
    assert L.qft_plan_create_uneven(ctypes.byref(h), None, 2, 0, 0) == \
        _lib.QFT_ERROR_INVALID_VALUE
    assert L.qft_plan_create_uneven(ctypes.byref(h), arr, 0, 0, 0) == \
        _lib.QFT_ERROR_INVALID_VALUE


def test_static_exec_rejects_before_any_hip_call():
    """qft_exec_fwd_static validates its arguments first (fake pointers are
    never touched): sizes beyond the static scratch give QFT_ERROR_SCRATCH."""
    L = _lib.lib()
    f = L.qft_exec_fwd_static
    p, q = 1 << 20, 1 << 40
    assert f(10, 4, 0, None, q, None) == _lib.QFT_ERROR_INVALID_VALUE
    assert f(10, 0, 0, p, q, None) == _lib.QFT_ERROR_INVALID_VALUE
    assert f(10, 4, 5, p, q, None) == _lib.QFT_ERROR_INVALID_VALUE
    assert f(0, 4, 0, p, q, None) == _lib.QFT_ERROR_INVALID_SIZE
    assert f(25, 1, 0, p, q, None) == _lib.QFT_ERROR_INVALID_SIZE
    assert f(17, 1, 0, p, q, None) == _lib.QFT_ERROR_SCRATCH
    assert f(16, 128, 0, p, q, None) == _lib.QFT_ERROR_SCRATCH   # 2^23 > 2^23 - 2^14
    assert f(15, 256, 1, p, q, None) == _lib.QFT_ERROR_SCRATCH
    assert f(16, 4, 0, p + 4, q, None) == _lib.QFT_ERROR_ALIGNMENT
    assert f(16, 4, 0, p, p + 64, None) == _lib.QFT_ERROR_OVERLAP


def test_fixed_point_plan_rejects():
    """QFT_I32 (fixed point) is a uniform-plan dtype for log2n <= 16."""
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.qft_plan_create(ctypes.byref(h), 17, 1, _lib.QFT_I32, 0) == \
        _lib.QFT_ERROR_INVALID_SIZE
    arr = (ctypes.c_int32 * 2)(4, 5)
    assert L.qft_plan_create_uneven(ctypes.byref(h), arr, 2, _lib.QFT_I32, 0) == \
        _lib.QFT_ERROR_INVALID_VALUE
    assert L.qft_plan_create_real(ctypes.byref(h), 8, 2, _lib.QFT_I32, 0) == \
        _lib.QFT_ERROR_INVALID_VALUE
    assert L.qft_exec_fwd_static(8, 2, _lib.QFT_I32, 1 << 20, 1 << 40, None) == \
        _lib.QFT_ERROR_INVALID_VALUE


def test_exec_and_info_reject_null_plan():
    L = _lib.lib()
    assert L.qft_exec_fwd(None, 8, 8, None) == _lib.QFT_ERROR_INVALID_VALUE
    assert L.qft_exec_bwd(None, 8, 8, None) == _lib.QFT_ERROR_INVALID_VALUE
    assert L.qft_plan_info(None, None, None, None, None) == _lib.QFT_ERROR_INVALID_VALUE
    assert L.qft_plan_destroy(None) == _lib.QFT_SUCCESS


def test_secant_table_rejects():
    L = _lib.lib()
    buf = (ctypes.c_float * 4)()
    assert L.qft_secant_table(None, 5) == _lib.QFT_ERROR_INVALID_VALUE
    assert L.qft_secant_table(buf, 2) == _lib.QFT_ERROR_INVALID_SIZE
    assert L.qft_secant_table(buf, 25) == _lib.QFT_ERROR_INVALID_SIZE


def _f32_neighbors_ulps(a, exact):
    """Distance of float32 a from the exact value, in float32 ulps at a."""
    a = np.float32(a)
    ulp = float(np.spacing(a))
    return abs(float(a) - exact) / ulp


@pytest.mark.parametrize("log2n", [3, 6, 10, 14])
def test_secant_table_vs_mpmath(log2n):
    """Entry L + m = 1/(2 cos(pi (2m+1)/(4L))): Sec. 6.1's constants, each the
    secant 1/(2 cos(theta n)) of eq. qft_38A.  Every entry must be the
    correctly rounded FP32 value or within one ulp of it."""
    mpmath.mp.dps = 60
    N = 1 << log2n
    t = np.frombuffer(qft.qft_secant_table(log2n), dtype=np.float32)
    assert t.size == N // 4 and t[0] == 0.0
    worst = 0.0
    bad = 0
    L = 1
    while 2 * L <= N // 4:
        for m in range(L):
            exact = 1 / (2 * mpmath.cos(mpmath.pi * (2 * m + 1) / (4 * L)))
            cr = np.float32(float(exact))  # correctly rounded via FP64 (60-digit source)
            d = _f32_neighbors_ulps(t[L + m], float(exact))
            worst = max(worst, d)
            if t[L + m] != cr:
                bad += 1
        L *= 2
    assert worst <= 1.0
    # the FP64 evaluation rounds correctly almost always
    assert bad <= max(1, (N // 4) // 1000)


def test_secant_table_base_constant():
    """Entry 1 = 1/(2 cos(pi/4)) is the cos(2 pi/8) of the N = 8 base cases."""
    t = np.frombuffer(qft.qft_secant_table(5), dtype=np.float32)
    assert t[1] == np.float32(np.cos(np.pi / 4))
    # nested sizes: the table for a smaller N is a prefix of a larger one
    big = np.frombuffer(qft.qft_secant_table(12), dtype=np.float32)
    assert np.array_equal(big[:t.size], t)


def test_schedule_entry_points_reject_null_plan():
    L = _lib.lib()
    n, c = ctypes.c_int(), ctypes.c_int()
    assert L.qft_plan_schedules(None, ctypes.byref(n), ctypes.byref(c)) == \
        _lib.QFT_ERROR_INVALID_VALUE
    assert L.qft_plan_schedule_name(None, 0) is None
    assert L.qft_plan_set_schedule(None, 0) == _lib.QFT_ERROR_INVALID_VALUE
    ms = (ctypes.c_double * 4)()
    assert L.qft_plan_autotune(None, 8, 8, None, 5, ms, 4, ctypes.byref(c)) == \
        _lib.QFT_ERROR_INVALID_VALUE


def test_real_entry_points_reject_bad_arguments():
    L = _lib.lib()
    h = ctypes.c_void_p(1)
    assert L.qft_plan_create_real(None, 10, 4, 0, 0) == _lib.QFT_ERROR_INVALID_VALUE
    assert L.qft_plan_create_real(ctypes.byref(h), 0, 4, 0, 0) == _lib.QFT_ERROR_INVALID_SIZE
    assert h.value is None
    assert L.qft_plan_create_real(ctypes.byref(h), 25, 4, 0, 0) == _lib.QFT_ERROR_INVALID_SIZE
    assert L.qft_plan_create_real(ctypes.byref(h), 10, 0, 0, 0) == _lib.QFT_ERROR_INVALID_VALUE
    assert L.qft_plan_create_real(ctypes.byref(h), 10, 4, 5, 0) == _lib.QFT_ERROR_INVALID_VALUE
    assert L.qft_exec_rdft(None, 8, 8, None) == _lib.QFT_ERROR_INVALID_VALUE
    assert L.qft_exec_dct0_dst0(None, 8, None, 8, None, None) == _lib.QFT_ERROR_INVALID_VALUE
