"""Acceptance bounds shared by the parity tests (GPU result against the FP64
oracle on the same stored input).

Two bounds per signal:

* relative L2 (eq. qft_44 before averaging over signals):
  ||X - X_ref||_2 / ||X_ref||_2 <= tol, with tol = 1e-5 * log2 N for FP32
  arithmetic;
* every single bin: |X(k) - X_ref(k)| <= c(n) * tol * rms(X_ref) (+ the output
  rounding of FP16 storage, below).

Where c(n) comes from.  The FP32 result is the exact DFT plus the rounding
errors of every butterfly, pushed through the rest of the (linear) network;
each output bin collects the contributions of ~log2 N stages, so its error is
a sum of many small independent terms and is modelled as a circular complex
Gaussian with variance sigma_k^2.  The relative L2 measures the mean,
rho^2 = mean_k sigma_k^2 / rms(X_ref)^2, and the first bound keeps rho <= tol.
For a circular complex Gaussian, P(|e| > c sigma) = exp(-c^2), so over n bins
P(max_k |e_k| > c sigma) <= n exp(-c^2); c = sqrt(ln n + ln 1e9) makes a false
failure less likely than 1e-9 per signal.  The secant multiplies amplify the
rounding of some intermediate values more than others, so the bins need not
share one variance: allowing sigma_k^2 up to 4 times the mean doubles c.
Hence c(n) = 2 sqrt(ln n + ln 1e9): 10.5 for n = 2^10, 12.2 for n = 2^24.

What it catches that the L2 cannot: one wrong bin of a 2^23-point signal moves
the relative L2 by only ~1/sqrt(N) = 3.5e-4, but its bin error is ~1 (the bin's
own size, ~rms), far above c * tol ~ 3e-3.

Where the per-bin bound does not apply: a round trip bwd(fwd(x))/N compared
with x itself.  Its error is the forward's error pulled back to the input,
F^H e / N, and for this method that image is not spread: it concentrates on a
few input samples (n = 1, N/2 - 1, N/2 + 1, N - 1 and their neighbours) and
grows about twice per doubling of N, e.g. 3.3e-4 rms(x) at N = 2^16 against a
median of 2.8e-6.  An FP32 model of the recursion in numpy (the oracle's
operation order with FP32 values and secants) shows the same samples with the
same sizes as the GPU, so it is a property of the method's arithmetic (the
large secants near theta n = pi/2), not of the kernels.  The forward and the
adjoint outputs are each checked bin by bin against the oracle; the round trip
keeps the relative L2 bound only.

FP16 storage: the output is rounded to half precision, so bin k may further
differ by up to 2^-11 |X_ref(k)| (unit roundoff of each component); the FP32
arithmetic part keeps its own bound.
"""
import math

import numpy as np

from oracle import direct as D

__all__ = ["tol", "bin_factor", "check", "FP16_UNIT"]

FP16_UNIT = 2.0 ** -11
_LN_1E9 = math.log(1e9)


def tol(logn):
    """Relative-L2 target of FP32 arithmetic, 1e-5 * log2 N."""
    return 1e-5 * logn


def bin_factor(n_bins):
    return 2.0 * math.sqrt(math.log(max(int(n_bins), 2)) + _LN_1E9)


def check(got, ref, logn, fp16=False, l2_tol=None, what="", per_bin=True):
    """Asserts both bounds for every signal (last axis = bins) and returns the
    worst relative L2 and the worst bin error in units of its bound (0 when
    per_bin is False: only the relative L2 is checked)."""
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    t = tol(logn)
    lt = l2_tol if l2_tol is not None else (1e-3 if fp16 else t)
    rel = D.relative_l2(got, ref)
    assert rel.max() <= lt, f"{what}: relative L2 {rel.max():.3e} > {lt:.1e}"
    if not per_bin:
        return float(rel.max()), 0.0
    n = ref.shape[-1]
    rms = np.sqrt(np.mean(np.abs(ref) ** 2, axis=-1, keepdims=True))
    bound = np.broadcast_to(bin_factor(n) * t * rms, ref.shape)
    if fp16:
        bound = bound + FP16_UNIT * np.abs(ref)
    err = np.abs(got - ref)
    ratio = err / bound
    worst = float(ratio.max())
    if worst > 1.0:
        idx = np.unravel_index(int(np.argmax(ratio)), ratio.shape)
        raise AssertionError(
            f"{what}: bin {idx} off by {err[idx]:.3e} > bound {bound[idx]:.3e} "
            f"(c = {bin_factor(n):.2f}, tol = {t:.1e}, rms = {rms[idx[:-1]].item():.3e})")
    return float(rel.max()), worst
