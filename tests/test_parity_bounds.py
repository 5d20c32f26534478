"""The acceptance bounds of the parity tests, exercised on the CPU: an oracle
result with FP32-sized rounding noise passes, and planted mistakes that the
per-signal relative L2 alone lets through fail the per-bin bound."""
import numpy as np
import pytest

from oracle import build as OB
from oracle import direct as D
from tests import parity as PB


def _case(logn, seed, rho):
    rng = np.random.default_rng(seed)
    N = 1 << logn
    x = rng.standard_normal((2, N)) + 1j * rng.standard_normal((2, N))
    ref = OB.cdft(x)
    rms = np.sqrt(np.mean(np.abs(ref) ** 2, -1, keepdims=True))
    noise = (rng.standard_normal(ref.shape) + 1j * rng.standard_normal(ref.shape)) / np.sqrt(2)
    return ref, ref + rho * rms * noise


def test_bin_factor_values():
    assert PB.bin_factor(1 << 10) == pytest.approx(10.52, abs=0.01)
    assert PB.bin_factor(1 << 24) == pytest.approx(12.22, abs=0.01)


@pytest.mark.parametrize("logn", [10, 16])
def test_rounding_noise_at_the_tolerance_passes(logn):
    ref, got = _case(logn, 1, PB.tol(logn) * 0.9)
    PB.check(got, ref, logn)


@pytest.mark.parametrize("logn", [12, 16])
def test_planted_single_bin_mistakes_fail(logn):
    ref, got = _case(logn, 2, PB.tol(logn) * 0.2)
    N = 1 << logn
    bad = got.copy()
    bad[0, N // 3] *= 1.005  # one bin 0.5% off: the L2 moves by ~0.005/sqrt(N)
    assert D.relative_l2(bad, ref).max() < PB.tol(logn)  # the L2 alone passes it
    with pytest.raises(AssertionError):
        PB.check(bad, ref, logn)
    swap = got.copy()  # two neighbouring bins exchanged
    swap[1, [5, 6]] = swap[1, [6, 5]]
    with pytest.raises(AssertionError):
        PB.check(swap, ref, logn)


def test_fp16_output_rounding_allowance():
    logn = 12
    ref, got = _case(logn, 3, PB.tol(logn) * 0.5)
    r16 = (got.real.astype(np.float16).astype(np.float64) +
           1j * got.imag.astype(np.float16).astype(np.float64))
    PB.check(r16, ref, logn, fp16=True)
    with pytest.raises(AssertionError):  # the same rounding is too much for FP32
        PB.check(r16, ref, logn)
