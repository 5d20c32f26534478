"""ctypes binding of the C ABI declared in include/qft.h (same names).

Only argument marshalling happens here; every step of the transform runs in
the gfx950 kernels of libqft.so.  The library must have been built in-tree
(``python -m paper_1301_0763_amd.build``); loading fails loudly otherwise.
"""
import ctypes
import os

from . import build as _build

QFT_SUCCESS = 0
QFT_ERROR_INVALID_VALUE = 1
QFT_ERROR_INVALID_SIZE = 2
QFT_ERROR_ALIGNMENT = 3
QFT_ERROR_OVERLAP = 4
QFT_ERROR_ALLOC = 5
QFT_ERROR_HIP = 6
QFT_ERROR_UNSUPPORTED = 7
QFT_ERROR_SCRATCH = 8

QFT_C32 = 0
QFT_C16 = 1
QFT_I32 = 2
QFT_MAX_LOG2N = 24

_lib = None


class QFTError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = f"{where}: {qft_status_string(status)} (status {status})"
        if status == QFT_ERROR_HIP:
            msg += f", hipError {qft_last_hip_error()}"
        super().__init__(msg)


def lib():
    """The loaded libqft.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            raise ImportError(f"libqft.so not built at {path}; run "
                              "`python -m paper_1301_0763_amd.build`")
        L = ctypes.CDLL(path)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.qft_plan_create.argtypes = [ctypes.POINTER(vp), i32, i64, i32, i32]
        L.qft_plan_create_uneven.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int32),
                                             i64, i32, i32]
        L.qft_exec_fwd.argtypes = [vp, vp, vp, vp]
        L.qft_exec_bwd.argtypes = [vp, vp, vp, vp]
        L.qft_plan_destroy.argtypes = [vp]
        L.qft_plan_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                    ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
        L.qft_secant_table.argtypes = [ctypes.POINTER(ctypes.c_float), i32]
        L.qft_status_string.argtypes = [i32]
        L.qft_status_string.restype = ctypes.c_char_p
        L.qft_last_hip_error.argtypes = []
        L.qft_plan_schedules.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.qft_plan_schedule_name.argtypes = [vp, i32]
        L.qft_plan_schedule_name.restype = ctypes.c_char_p
        L.qft_plan_set_schedule.argtypes = [vp, i32]
        L.qft_plan_autotune.argtypes = [vp, vp, vp, vp, i32, ctypes.POINTER(ctypes.c_double), i32,
                                        ctypes.POINTER(i32)]
        L.qft_plan_create_real.argtypes = [ctypes.POINTER(vp), i32, i64, i32, i32]
        L.qft_exec_rdft.argtypes = [vp, vp, vp, vp]
        L.qft_exec_dct0_dst0.argtypes = [vp, vp, vp, vp, vp, vp]
        L.qft_exec_fwd_static.argtypes = [i32, i64, i32, vp, vp, vp]
        for f in ("qft_plan_create", "qft_plan_create_uneven", "qft_exec_fwd", "qft_exec_bwd",
                  "qft_plan_destroy", "qft_plan_info", "qft_secant_table",
                  "qft_last_hip_error", "qft_plan_schedules", "qft_plan_set_schedule",
                  "qft_plan_autotune", "qft_plan_create_real", "qft_exec_rdft",
                  "qft_exec_dct0_dst0", "qft_exec_fwd_static"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status, where):
    if status != QFT_SUCCESS:
        raise QFTError(status, where)


def qft_status_string(status):
    return lib().qft_status_string(int(status)).decode()


def qft_last_hip_error():
    return lib().qft_last_hip_error()


def qft_plan_create(log2n, batch, dtype=QFT_C32, device=0):
    """Returns an opaque plan handle (int)."""
    h = ctypes.c_void_p()
    _check(lib().qft_plan_create(ctypes.byref(h), int(log2n), int(batch), int(dtype),
                                 int(device)), "qft_plan_create")
    return h.value


def qft_plan_create_uneven(log2n_list, dtype=QFT_C32, device=0):
    arr = (ctypes.c_int32 * len(log2n_list))(*[int(v) for v in log2n_list])
    h = ctypes.c_void_p()
    _check(lib().qft_plan_create_uneven(ctypes.byref(h), arr, len(log2n_list), int(dtype),
                                        int(device)), "qft_plan_create_uneven")
    return h.value


def qft_exec_fwd(plan, in_ptr, out_ptr, stream=0):
    _check(lib().qft_exec_fwd(plan, in_ptr, out_ptr, stream), "qft_exec_fwd")


def qft_exec_fwd_static(log2n, batch, dtype, in_ptr, out_ptr, stream=0):
    """Plan-free forward transform on the current device using the library's
    static scratch (no device allocation; see include/qft.h)."""
    _check(lib().qft_exec_fwd_static(int(log2n), int(batch), int(dtype), in_ptr, out_ptr,
                                     stream), "qft_exec_fwd_static")


def qft_exec_bwd(plan, in_ptr, out_ptr, stream=0):
    _check(lib().qft_exec_bwd(plan, in_ptr, out_ptr, stream), "qft_exec_bwd")


def qft_plan_destroy(plan):
    _check(lib().qft_plan_destroy(plan), "qft_plan_destroy")


def qft_plan_info(plan):
    tp, ab = ctypes.c_int64(), ctypes.c_int64()
    f5, fa = ctypes.c_double(), ctypes.c_double()
    _check(lib().qft_plan_info(plan, ctypes.byref(tp), ctypes.byref(ab), ctypes.byref(f5),
                               ctypes.byref(fa)), "qft_plan_info")
    return dict(total_points=tp.value, algo_bytes=ab.value, flops_5nlogn=f5.value,
                flops_actual=fa.value)


def qft_secant_table(log2n_max):
    """Host-side FP32 constant table (N/4 entries) as a list-like ctypes array."""
    n = (1 << int(log2n_max)) // 4 if log2n_max >= 3 else 2
    buf = (ctypes.c_float * n)()
    _check(lib().qft_secant_table(buf, int(log2n_max)), "qft_secant_table")
    return buf


def qft_plan_schedules(plan):
    """(number of schedules, index exec uses)."""
    n, c = ctypes.c_int(), ctypes.c_int()
    _check(lib().qft_plan_schedules(plan, ctypes.byref(n), ctypes.byref(c)),
           "qft_plan_schedules")
    return n.value, c.value


def qft_plan_schedule_name(plan, schedule):
    name = lib().qft_plan_schedule_name(plan, int(schedule))
    if name is None:
        raise QFTError(QFT_ERROR_INVALID_VALUE, "qft_plan_schedule_name")
    return name.decode()


def qft_plan_set_schedule(plan, schedule):
    _check(lib().qft_plan_set_schedule(plan, int(schedule)), "qft_plan_set_schedule")


def qft_plan_autotune(plan, in_ptr, out_ptr, stream=0, reps=10):
    """Times every schedule; returns (chosen index, [ms per schedule])."""
    n, _ = qft_plan_schedules(plan)
    ms = (ctypes.c_double * max(n, 1))()
    chosen = ctypes.c_int()
    _check(lib().qft_plan_autotune(plan, in_ptr, out_ptr, stream, int(reps), ms, n,
                                   ctypes.byref(chosen)), "qft_plan_autotune")
    return chosen.value, [ms[i] for i in range(n)]


def qft_plan_create_real(log2n, batch, dtype=QFT_C32, device=0):
    """Real-input plan for `batch` real signals of 2^log2n points."""
    h = ctypes.c_void_p()
    _check(lib().qft_plan_create_real(ctypes.byref(h), int(log2n), int(batch), int(dtype),
                                      int(device)), "qft_plan_create_real")
    return h.value


def qft_exec_rdft(plan, in_ptr, out_ptr, stream=0):
    _check(lib().qft_exec_rdft(plan, in_ptr, out_ptr, stream), "qft_exec_rdft")


def qft_exec_dct0_dst0(plan, c_ptr, d_ptr, C_ptr, S_ptr, stream=0):
    """Null (None/0) pointers leave out the DCT-0 or the DST-0."""
    _check(lib().qft_exec_dct0_dst0(plan, c_ptr or None, d_ptr or None, C_ptr or None,
                                    S_ptr or None, stream), "qft_exec_dct0_dst0")
