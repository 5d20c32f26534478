"""Builds the C oracle (``qft_ref.c``) into ``oracle/libqft_ref.so``.

Test infrastructure only.  Flags: -O2, no fast-math, -ffp-contract=off (no
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
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
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


if __name__ == "__main__":
    print(build())
