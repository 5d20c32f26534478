"""Improved-QFT power-of-two DFT on MI355X (gfx950).

Python face of the C ABI in include/qft.h.  PyTorch is used only for device
memory and streams: tensors are handed to the library as raw device pointers
on torch's current HIP stream, and every arithmetic step runs in the library's
gfx950 kernels.

    X = fft(x)              # X(k) = sum_n x(n) exp(-2 pi i n k / N), last axis
    x = fft_adjoint(X)      # conjugate transpose, unnormalised
    X = QFTFunction.apply(x)            # differentiable (backward = adjoint)
    Y = fft_packed(values, log2n_list)  # uneven batch, one persistent launch
    H = rdft(xr)            # real input [..., N] -> half spectrum [..., N/2+1]
    C = dct0(c); S = dst0(d)            # DCT-0 / DST-0 of periodization N

Supported storage: complex64 (FP32) and complex32 / torch.chalf (FP16 storage,
FP32 arithmetic).  N = 2^r with 1 <= r <= 24.
"""
import collections
import threading

from . import _lib
from ._lib import (QFT_C16, QFT_C32, QFT_I32, QFT_MAX_LOG2N, QFTError, qft_exec_bwd,
                   qft_exec_dct0_dst0, qft_exec_fwd, qft_exec_fwd_static, qft_exec_rdft,
                   qft_last_hip_error,
                   qft_plan_autotune, qft_plan_create, qft_plan_create_real,
                   qft_plan_create_uneven, qft_plan_destroy, qft_plan_info,
                   qft_plan_schedule_name, qft_plan_schedules, qft_plan_set_schedule,
                   qft_secant_table, qft_status_string)

__all__ = [
    "Plan", "UnevenPlan", "fft", "fft_adjoint", "fft_packed", "QFTFunction", "QFTError",
    "qft_plan_create", "qft_plan_create_uneven", "qft_exec_fwd", "qft_exec_bwd",
    "qft_plan_destroy", "qft_plan_info", "qft_secant_table", "qft_status_string",
    "qft_last_hip_error", "qft_plan_schedules", "qft_plan_schedule_name",
    "qft_plan_set_schedule", "qft_plan_autotune", "qft_plan_create_real", "qft_exec_rdft",
    "qft_exec_dct0_dst0", "qft_exec_fwd_static", "RealPlan", "rdft", "dct0", "dst0",
    "QFT_C32", "QFT_C16", "QFT_I32", "QFT_MAX_LOG2N", "FixedPlan", "fft_fixed",
]


def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.complex64:
        return QFT_C32
    if t.dtype == torch.complex32:
        return QFT_C16
    raise TypeError(f"unsupported dtype {t.dtype}; use complex64 or complex32")


def _log2n(N):
    r = int(N).bit_length() - 1
    if N < 2 or (1 << r) != N:
        raise ValueError(f"transform length {N} is not a power of two >= 2")
    return r


def _stream_ptr(device):
    return _torch().cuda.current_stream(device).cuda_stream


class Plan:
    """Plan for `batch` transforms of length 2^log2n (qft_plan_create)."""

    def __init__(self, log2n, batch, dtype=QFT_C32, device=0):
        self.log2n, self.batch, self.dtype, self.device = int(log2n), int(batch), dtype, device
        self.handle = qft_plan_create(log2n, batch, dtype, device)
        self.info = qft_plan_info(self.handle)

    def _check(self, x, y):
        if not (x.is_cuda and y.is_cuda):
            raise ValueError("tensors must be on the GPU")
        if not (x.is_contiguous() and y.is_contiguous()):
            raise ValueError("tensors must be contiguous")
        if x.numel() != self.info["total_points"] or y.numel() != self.info["total_points"]:
            raise ValueError("tensor size does not match the plan")
        if _dtype_code(x) != self.dtype or _dtype_code(y) != self.dtype:
            raise ValueError("tensor dtype does not match the plan")

    def forward(self, x, out=None):
        torch = _torch()
        out = torch.empty_like(x) if out is None else out
        self._check(x, out)
        qft_exec_fwd(self.handle, x.data_ptr(), out.data_ptr(), _stream_ptr(x.device))
        return out

    def adjoint(self, X, out=None):
        torch = _torch()
        out = torch.empty_like(X) if out is None else out
        self._check(X, out)
        qft_exec_bwd(self.handle, X.data_ptr(), out.data_ptr(), _stream_ptr(X.device))
        return out

    @property
    def schedules(self):
        """Names of the plan's schedules (index = schedule number)."""
        n, _ = qft_plan_schedules(self.handle)
        return [qft_plan_schedule_name(self.handle, i) for i in range(n)]

    @property
    def schedule(self):
        """Index of the schedule exec uses."""
        return qft_plan_schedules(self.handle)[1]

    @schedule.setter
    def schedule(self, index):
        qft_plan_set_schedule(self.handle, index)

    def autotune(self, x, out=None, reps=10):
        """Times every schedule on x (result written to out) and keeps the
        fastest; returns {name: ms}.  Synchronises the current stream."""
        torch = _torch()
        out = torch.empty_like(x) if out is None else out
        self._check(x, out)
        _, ms = qft_plan_autotune(self.handle, x.data_ptr(), out.data_ptr(),
                                  _stream_ptr(x.device), reps)
        return dict(zip(self.schedules, ms))

    def close(self):
        if self.handle:
            qft_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class UnevenPlan(Plan):
    """Plan for transforms of lengths 2^log2n[i] packed back to back."""

    def __init__(self, log2n_list, dtype=QFT_C32, device=0):
        self.log2n_list = [int(v) for v in log2n_list]
        self.dtype, self.device = dtype, device
        self.handle = qft_plan_create_uneven(self.log2n_list, dtype, device)
        self.info = qft_plan_info(self.handle)


class FixedPlan:
    """Fixed-point plan (qft_plan_create with QFT_I32): `batch` transforms of
    2^log2n points, complex int32 pairs as int32 tensors [..., N, 2]."""

    def __init__(self, log2n, batch, device=0):
        self.log2n, self.batch, self.device = int(log2n), int(batch), device
        self.handle = qft_plan_create(log2n, batch, QFT_I32, device)
        self.info = qft_plan_info(self.handle)

    def _check(self, x, y):
        torch = _torch()
        for t in (x, y):
            if not (t.is_cuda and t.is_contiguous() and t.dtype == torch.int32):
                raise ValueError("tensors must be contiguous int32 GPU tensors")
            if t.numel() != 2 * self.info["total_points"]:
                raise ValueError("tensor size does not match the plan")

    def forward(self, x, out=None):
        torch = _torch()
        out = torch.empty_like(x) if out is None else out
        self._check(x, out)
        qft_exec_fwd(self.handle, x.data_ptr(), out.data_ptr(), _stream_ptr(x.device))
        return out

    def adjoint(self, X, out=None):
        torch = _torch()
        out = torch.empty_like(X) if out is None else out
        self._check(X, out)
        qft_exec_bwd(self.handle, X.data_ptr(), out.data_ptr(), _stream_ptr(X.device))
        return out

    def close(self):
        if self.handle:
            qft_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _real_code(t):
    torch = _torch()
    if t.dtype == torch.float32:
        return QFT_C32
    if t.dtype == torch.float16:
        return QFT_C16
    raise TypeError(f"unsupported dtype {t.dtype}; use float32 or float16")


class RealPlan:
    """Real-input plan (qft_plan_create_real): `batch` real signals of 2^log2n
    points; rdft and DCT-0/DST-0 execs."""

    def __init__(self, log2n, batch, dtype=QFT_C32, device=0):
        self.log2n, self.batch, self.dtype, self.device = int(log2n), int(batch), dtype, device
        self.handle = qft_plan_create_real(log2n, batch, dtype, device)
        self.info = qft_plan_info(self.handle)

    def _rows(self, t, length, what):
        if not (t.is_cuda and t.is_contiguous()):
            raise ValueError(f"{what} must be a contiguous GPU tensor")
        if t.numel() != self.batch * length or _real_code(t) != self.dtype:
            raise ValueError(f"{what}: expected {self.batch} x {length} reals of the plan's dtype")

    def rdft(self, x, out=None):
        torch = _torch()
        N = 1 << self.log2n
        self._rows(x, N, "x")
        cdt = torch.complex64 if self.dtype == QFT_C32 else torch.complex32
        shape = tuple(x.shape[:-1]) + (N // 2 + 1,)
        out = torch.empty(shape, dtype=cdt, device=x.device) if out is None else out
        if not (out.is_contiguous() and out.numel() == self.batch * (N // 2 + 1)):
            raise ValueError("out: expected batch x (N/2 + 1) complex values")
        qft_exec_rdft(self.handle, x.data_ptr(), out.data_ptr(), _stream_ptr(x.device))
        return out

    def dct0_dst0(self, c=None, d=None):
        """(C, S) for the given inputs; a missing input gives None."""
        torch = _torch()
        h = (1 << self.log2n) // 2
        if c is None and d is None:
            raise ValueError("give c, d or both")
        if h - 1 == 0:
            d = None
        ref = c if c is not None else d
        C = S = None
        if c is not None:
            self._rows(c, h + 1, "c")
            C = torch.empty_like(c)
        if d is not None:
            self._rows(d, h - 1, "d")
            S = torch.empty_like(d)
        qft_exec_dct0_dst0(self.handle, c.data_ptr() if c is not None else None,
                           d.data_ptr() if d is not None else None,
                           C.data_ptr() if C is not None else None,
                           S.data_ptr() if S is not None else None, _stream_ptr(ref.device))
        return C, S

    def close(self):
        if self.handle:
            qft_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Plans made by the convenience functions below.  A plan owns scratch memory
# that one exec uses at a time (qft.h), so a cached plan serves one stream:
# the stream is part of the key, and execs on two streams never share one.
_cache = {}
_cache_lock = threading.Lock()
_PACKED_MAX = 4
_packed = collections.OrderedDict()  # uneven plans, least recently used first


def _dev_index(t):
    return t.device.index if t.device.index is not None else _torch().cuda.current_device()


def _real_plan(log2n, rows, t):
    dev = _dev_index(t)
    key = ("real", log2n, rows, _real_code(t), dev, _stream_ptr(t.device))
    with _cache_lock:
        p = _cache.get(key)
        if p is None:
            p = RealPlan(log2n, rows, key[3], dev)
            _cache[key] = p
    return p


def rdft(x):
    """Half spectrum X(k), k = 0..N/2, of the real signals on the last axis."""
    x = x.contiguous()
    N = x.shape[-1]
    return _real_plan(_log2n(N), x.numel() // N, x).rdft(x)


def dct0(c):
    """DCT-0 of periodization N of c(n), n = 0..N/2 (last axis of N/2 + 1)."""
    c = c.contiguous()
    N = 2 * (c.shape[-1] - 1)
    return _real_plan(_log2n(N), c.numel() // c.shape[-1], c).dct0_dst0(c=c)[0]


def dst0(d):
    """DST-0 of periodization N of d(n), n = 1..N/2-1 (last axis of N/2 - 1)."""
    d = d.contiguous()
    N = 2 * (d.shape[-1] + 1)
    return _real_plan(_log2n(N), d.numel() // d.shape[-1], d).dct0_dst0(d=d)[1]


def _plan_for(x):
    N = x.shape[-1]
    log2n = _log2n(N)
    batch = x.numel() // N
    dev = _dev_index(x)
    key = (log2n, batch, _dtype_code(x), dev, _stream_ptr(x.device))
    with _cache_lock:
        p = _cache.get(key)
        if p is None:
            p = Plan(log2n, batch, key[2], dev)
            _cache[key] = p
    return p


def fft_fixed(x):
    """Fixed-point forward transform of int32 tensors [..., N, 2] (re, im)."""
    x = x.contiguous()
    N = x.shape[-2]
    log2n = _log2n(N)
    dev = _dev_index(x)
    key = ("fixed", log2n, x.numel() // (2 * N), dev, _stream_ptr(x.device))
    with _cache_lock:
        p = _cache.get(key)
        if p is None:
            p = FixedPlan(log2n, key[2], dev)
            _cache[key] = p
    return p.forward(x)


def fft(x):
    """Forward unnormalised DFT of the last axis of a complex GPU tensor."""
    x = x.contiguous()
    return _plan_for(x).forward(x)


def fft_adjoint(X):
    """Adjoint (conjugate-transpose) DFT of the last axis: fft_adjoint(fft(x)) = N x."""
    X = X.contiguous()
    return _plan_for(X).adjoint(X)


def fft_packed(values, log2n_list, plan=None):
    """Forward DFTs of an uneven batch packed back to back in a 1-D tensor.
    Without `plan`, the plan is kept for later calls with the same sizes, dtype,
    device and stream (the last few such lists)."""
    values = values.contiguous()
    if plan is None:
        dev = _dev_index(values)
        key = (tuple(int(v) for v in log2n_list), _dtype_code(values), dev,
               _stream_ptr(values.device))
        with _cache_lock:
            plan = _packed.get(key)
            if plan is None:
                plan = UnevenPlan(key[0], key[1], dev)
                _packed[key] = plan
                while len(_packed) > _PACKED_MAX:
                    _, old = _packed.popitem(last=False)
                    # the evicted plan's last exec may still run on its stream
                    _torch().cuda.synchronize(old.device)
                    old.close()
            else:
                _packed.move_to_end(key)
    return plan.forward(values)


class QFTFunction(_torch().autograd.Function):
    """X = F x with backward F^H g (PyTorch's convention for C -> C maps: the
    vector-Jacobian product of a linear map is its adjoint), both through the
    same improved-QFT plan."""

    @staticmethod
    def forward(ctx, x):
        return fft(x)

    @staticmethod
    def backward(ctx, g):
        return fft_adjoint(g.contiguous())
