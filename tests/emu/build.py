"""Builds the CPU emulation of the GPU kernels (tests/emu/libqft_emu.so).

Host-only hipcc build (no device code) of qft_emu.cpp, which includes the
library's kernel bodies and schedules unchanged.  -O0 keeps the template-heavy
build to seconds; the emulated problems are small.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "qft_emu.cpp")
LIB = os.path.join(HERE, "libqft_emu.so")
DEPS = [SRC] + [os.path.join(ROOT, "paper_1301_0763_amd", "csrc", f)
                for f in ("qft_device.hpp", "qft_schedule.hpp", "qft_cache.hpp",
                          "qft_fixed.hpp")]


def build(force=True):
    if not force and os.path.exists(LIB) and \
            all(os.path.getmtime(d) <= os.path.getmtime(LIB) for d in DEPS):
        return LIB
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc"
    cmd = [hipcc, "-x", "hip", "--offload-host-only", "-O0", "-std=c++20", "-fPIC", "-shared",
           SRC, "-o", LIB + ".tmp", "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def load():
    import ctypes
    L = ctypes.CDLL(build(force=False))
    i, vp, i64 = ctypes.c_int, ctypes.c_void_p, ctypes.c_int64
    L.emu_multipass.argtypes = [i, i, vp, vp, i, i64, i, i]
    L.emu_uneven.argtypes = [i, i, vp, vp, ctypes.POINTER(ctypes.c_int32), i64, i, i]
    L.emu_twopass.argtypes = [i, i, vp, vp, i, i64, i64]
    L.emu_tile_s.argtypes = [i, i, vp, vp, i, i, vp]
    L.emu_tile_p.argtypes = [i, i, vp, vp, i, i64, i64]
    L.emu_tile_pg.argtypes = [i, i, vp, vp, i, vp, vp, i64, i64]
    L.emu_tile_real.argtypes = [i, i, i, i64, vp, vp, vp, vp]
    L.emu_multipass_real.argtypes = [i, i, i, i64, vp, vp, vp, vp, i, i]
    L.emu_race_model_check.argtypes = [i, i]
    L.emu_multipass_levels.argtypes = [i, vp, vp, i, i64, i, i, i, i, i]
    cp = ctypes.c_char_p
    L.emu_cache_store.argtypes = [cp, cp, cp]
    L.emu_cache_lookup.argtypes = [cp, cp, ctypes.c_char_p, i]
    L.emu_cache_path.argtypes = [ctypes.c_char_p, i]
    L.emu_fixed.argtypes = [vp, vp, i, i64, i, i]
    L.emu_fixed_table.argtypes = [i, vp, vp]
    for f in (L.emu_multipass, L.emu_uneven, L.emu_twopass, L.emu_tile_s, L.emu_tile_p,
              L.emu_tile_pg,
              L.emu_tile_real, L.emu_multipass_real, L.emu_race_model_check,
              L.emu_multipass_levels, L.emu_cache_store, L.emu_cache_lookup, L.emu_cache_path,
              L.emu_fixed, L.emu_fixed_table):
        f.restype = i
    return L


if __name__ == "__main__":
    print(build())
