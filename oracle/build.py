"""Builds the C oracle (``qft_ref.c``) into ``oracle/libqft_ref.so``.

Test infrastructure only.  Flags: -O3, no fast-math, -ffp-contract=off (no
multiply-add fusion, matching the FP64 numpy oracle), OpenMP over the batch.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qft_ref.c")
LIB = os.path.join(HERE, "libqft_ref.so")


def build(force=True):
    """Compile the C oracle; returns the path of the shared library."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    cmd = ["gcc", "-O3", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
           "-shared", "-std=c11", "-D_DEFAULT_SOURCE", SRC, "-o", LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def load():
    """Build if needed and return the ctypes handle with typed entry points."""
    import ctypes
    lib = ctypes.CDLL(build(force=False))
    lib.qft_ref_cdft.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int64]
    lib.qft_ref_cdft.restype = ctypes.c_int
    lib.qft_ref_threads.argtypes = []
    lib.qft_ref_threads.restype = ctypes.c_int
    lib.qft_ref_dct_dst.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                    ctypes.c_int64, ctypes.c_int]
    lib.qft_ref_dct_dst.restype = ctypes.c_int
    lib.qft_ref_set_threads.argtypes = [ctypes.c_int]
    lib.qft_ref_set_threads.restype = None
    return lib


def cdft(x):
    """Forward CDFT of the last axis of complex array x through the C oracle."""
    import numpy as np
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    N = x.shape[-1]
    r = N.bit_length() - 1
    if N < 2 or (1 << r) != N:
        raise ValueError("N must be a power of two >= 2")
    out = np.empty_like(x)
    lib = load()
    st = lib.qft_ref_cdft(x.ctypes.data, out.ctypes.data, r, x.size // N)
    if st != 0:
        raise RuntimeError(f"qft_ref_cdft failed with {st}")
    return out


def _dct_dst(s, N, dst_side):
    import numpy as np
    s = np.ascontiguousarray(np.asarray(s, dtype=np.float64))
    r = int(N).bit_length() - 1
    if N < 2 or (1 << r) != N:
        raise ValueError("N must be a power of two >= 2")
    length = N // 2 - 1 if dst_side else N // 2 + 1
    if s.shape[-1] != length:
        raise ValueError(f"expected {length} samples per signal, got {s.shape[-1]}")
    out = np.empty_like(s)
    st = load().qft_ref_dct_dst(s.ctypes.data, out.ctypes.data, r, s.size // length,
                                1 if dst_side else 0)
    if st != 0:
        raise RuntimeError(f"qft_ref_dct_dst failed with {st}")
    return out


def dct(c, N):
    """DCT-0 of s_dc_tt (last axis, N/2+1 samples) through the C oracle."""
    return _dct_dst(c, N, False)


def dst(d, N):
    """DST-0 of s_ds_tt (last axis, N/2-1 samples) through the C oracle."""
    return _dct_dst(d, N, True)


def set_threads(n):
    """OpenMP threads for later calls (n >= 1)."""
    load().qft_ref_set_threads(int(n))


def threads():
    return load().qft_ref_threads()


if __name__ == "__main__":
    print(build())
