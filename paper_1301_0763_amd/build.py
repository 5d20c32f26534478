"""Builds the gfx950 library ``libqft.so`` in-tree from ``csrc/qft_lib.hip``.

Flags: ``--offload-arch=gfx950 -O3`` and packed FP32 instructions disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``; the host pass warns
that it does not know the feature, which is harmless).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "qft_lib.hip")
DEPS = [SRC] + [os.path.join(HERE, "csrc", f) for f in ("qft_device.hpp", "qft_schedule.hpp")]
LIB = os.path.join(HERE, "libqft.so")
ROOT = os.path.dirname(HERE)
HEADER = os.path.join(ROOT, "include", "qft.h")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def build(verbose=False):
    """Compile libqft.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + HIPCC_FLAGS + [SRC, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    msgs = [l for l in (res.stdout + res.stderr).splitlines() if noise not in l]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs), file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


def stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS + [HEADER])


if __name__ == "__main__":
    print(build(verbose=True))
