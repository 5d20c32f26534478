"""Builds the gfx950 library ``libqft.so`` in-tree.

Twenty-four translation units compile in parallel (at most MAX_JOBS or one
per CPU at a time) and link into one shared library: ``csrc/qft_lib.hip``
(plans, C ABI, two-pass kernels), ``csrc/qft_fixed.hip`` (the fixed-point
kernels), ``csrc/qft_multipass.hip`` once per
storage type (``-DQFT_MP_DT=0`` complex FP32, ``=1`` complex FP16) and
``csrc/qft_tiles.hip`` once per storage type (``-DQFT_TILE_DT``), tile size
(``-DQFT_TILE_TL=10 .. 14``) and direction (``-DQFT_TILE_SWAP=0`` forward,
``=1`` adjoint).

Flags: ``--offload-arch=gfx950 -O3 -ffp-contract=off`` and packed FP32 instructions disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``; the host pass warns
that it does not know the feature, which is harmless).
"""
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SRC = os.path.join(CSRC, "qft_lib.hip")
TILES = os.path.join(CSRC, "qft_tiles.hip")
MULTI = os.path.join(CSRC, "qft_multipass.hip")
FIXED = os.path.join(CSRC, "qft_fixed.hip")
DEPS = [SRC, TILES, MULTI, FIXED] + [os.path.join(CSRC, f) for f in
                       ("qft_device.hpp", "qft_schedule.hpp", "qft_kernels.hpp",
                        "qft_cache.hpp", "qft_fixed.hpp")]
LIB = os.path.join(HERE, "libqft.so")
ROOT = os.path.dirname(HERE)
HEADER = os.path.join(ROOT, "include", "qft.h")

# -ffp-contract=off: every kernel rounds each product and sum as written,
# so the same transform gives bit-identical results in every kernel that
# computes it (uniform, uneven and real-input tiles, any schedule), whatever
# the surrounding code lets the optimiser fuse.
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
NOISE = "is not a recognized feature for this target"


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def build(verbose=False):
    """Compile libqft.so (always recompiles)."""
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="qft_build_") as tmp:
        units = [(TILES, ["-DQFT_TILE_DT=%d" % dt, "-DQFT_TILE_TL=%d" % tl,
                          "-DQFT_TILE_SWAP=%d" % sw], "tiles_%d_%d_%d.o" % (dt, tl, sw))
                 for tl in (14, 13, 12, 11, 10) for dt in (0, 1) for sw in (0, 1)]
        units[0:0] = [(SRC, [], "lib.o"), (FIXED, [], "fixed.o")] + [
            (MULTI, ["-DQFT_MP_DT=%d" % dt], "multipass_%d.o" % dt) for dt in (0, 1)]
        # at most one compiler per CPU (each takes ~1-2 GB)
        jobs = max(1, min(len(units), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
        msgs, failed, running, pending = [], False, [], list(units)
        while pending or running:
            while pending and len(running) < jobs:
                src, defs, obj = pending.pop(0)
                cmd = [cc] + HIPCC_FLAGS + defs + ["-c", src, "-o", os.path.join(tmp, obj)]
                running.append(subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.STDOUT, text=True))
            pr = running.pop(0)
            out, _ = pr.communicate()
            msgs += [l for l in out.splitlines() if NOISE not in l]
            failed |= pr.returncode != 0
        if failed:
            raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
        out_tmp = LIB + ".tmp"
        link = [cc, "--offload-arch=gfx950", "-shared", "-fPIC"] + \
            [os.path.join(tmp, u[2]) for u in units] + ["-o", out_tmp]
        res = subprocess.run(link, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    if verbose and msgs:
        print("\n".join(msgs), file=sys.stderr)
    os.replace(out_tmp, LIB)
    return LIB


def stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS + [HEADER])


if __name__ == "__main__":
    print(build(verbose=True))
