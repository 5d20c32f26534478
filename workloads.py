"""Seeded synthetic inputs for the improved-QFT transform.

This module only draws random numbers; it holds none of the transform's
arithmetic.  The tests, the benchmark and the smoke check all take their
inputs from here and hand the same arrays to the GPU library and to the CPU
oracle.

Conventions: numpy PCG64 (``default_rng(seed)``); values are drawn in FP64 and
rounded once (round-to-nearest-even) to the storage type; within a draw all
real parts come first, then all imaginary parts, in C order over [B, N] (or
over the packed buffer of an uneven batch).

The paper's own accuracy experiment uses random complex signals with real and
imaginary parts uniform in (-0.5, 0.5) (Sec. 6.3); the workloads below are
that family (scaled), Gaussian signals, and a sum of exact-bin tones plus
noise.  There is no dataset; every workload is synthetic.
"""
import numpy as np

__all__ = ["uniform", "normal", "tones", "uneven_sizes", "WORKLOADS", "make"]


def _complex(re, im, dtype):
    out = np.empty(re.shape, np.complex64 if dtype == np.float32 else np.complex128)
    out.real = re.astype(dtype)
    out.imag = im.astype(dtype)
    return out


def uniform(seed, shape, lo=-1.0, hi=1.0, dtype=np.float32):
    rng = np.random.default_rng(seed)
    re = rng.uniform(lo, hi, shape)
    im = rng.uniform(lo, hi, shape)
    return _complex(re, im, dtype)


def normal(seed, shape, dtype=np.float32):
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return _complex(re, im, dtype)


def tones(seed, N, ntones=8, amp=(0.1, 1.0), noise=1e-3, dtype=np.float32):
    """x(n) = sum_i a_i exp(+2 pi i f_i n / N) + noise, f_i distinct integer
    bins drawn uniformly in [0, N), a_i ~ U[amp], noise re/im ~ N(0, noise^2).
    Returns (x [1, N], freqs, amps).  The angle index f_i n is reduced
    exactly (mod N) in integers before the FP64 exponential."""
    rng = np.random.default_rng(seed)
    freqs = []
    while len(freqs) < ntones:
        f = int(rng.integers(0, N))
        if f not in freqs:
            freqs.append(f)
    amps = rng.uniform(amp[0], amp[1], ntones)
    n = np.arange(N, dtype=np.int64)
    re = np.zeros(N)
    im = np.zeros(N)
    for f, a in zip(freqs, amps):
        ang = (2.0 * np.pi / N) * ((f * n) % N)
        re += a * np.cos(ang)
        im += a * np.sin(ang)
    re += rng.normal(0.0, noise, N)
    im += rng.normal(0.0, noise, N)
    return _complex(re[None], im[None], dtype), np.array(freqs), amps


def uneven_sizes(seed, count, rmin, rmax):
    """log2 sizes r ~ U{rmin..rmax} for `count` transforms, then the packed
    values re/im ~ U[-1, 1] (drawn from the same generator, sizes first)."""
    rng = np.random.default_rng(seed)
    r = rng.integers(rmin, rmax + 1, count).astype(np.int32)
    total = int(np.sum(np.int64(1) << r.astype(np.int64)))
    re = rng.uniform(-1.0, 1.0, total)
    im = rng.uniform(-1.0, 1.0, total)
    return r, _complex(re, im, np.float32)


# The five workload configurations (seeds 0..4).
WORKLOADS = {
    "c1": dict(desc="N=2^10, batch 64, re/im ~ U[-1,1], seed 0", log2n=10, batch=64),
    "c2": dict(desc="N=2^16, batch 256, re/im ~ N(0,1), seed 1", log2n=16, batch=256),
    "c3": dict(desc="N=2^24, batch 1, 8 exact-bin tones (a ~ U[0.1,1]) + N(0,1e-3) noise, seed 2",
               log2n=24, batch=1),
    "c4": dict(desc="4096 transforms, N=2^r, r ~ U{6..14}, re/im ~ U[-1,1], seed 3",
               count=4096, rmin=6, rmax=14),
    "c5": dict(desc="N=4096, batch 512, x re/im ~ U[-1,1] then w ~ U[0,1], seed 4",
               log2n=12, batch=512),
}


def make(name):
    """Input arrays of a named workload (see WORKLOADS)."""
    w = WORKLOADS[name]
    if name == "c1":
        return uniform(0, (w["batch"], 1 << w["log2n"]))
    if name == "c2":
        return normal(1, (w["batch"], 1 << w["log2n"]))
    if name == "c3":
        return tones(2, 1 << w["log2n"])
    if name == "c4":
        return uneven_sizes(3, w["count"], w["rmin"], w["rmax"])
    if name == "c5":
        rng = np.random.default_rng(4)
        shape = (w["batch"], 1 << w["log2n"])
        re = rng.uniform(-1.0, 1.0, shape)
        im = rng.uniform(-1.0, 1.0, shape)
        wgt = rng.uniform(0.0, 1.0, shape).astype(np.float32)
        return _complex(re, im, np.float32), wgt
    raise KeyError(name)
