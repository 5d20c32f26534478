"""Pins for Oracle F, the fixed-point improved QFT (oracle/qft_fixed.py).

* structure: the same code on FP64 values with exact products equals the FP64
  oracle (oracle/qft.py) to rounding, for every size;
* hand-worked integer results (tests/golden/fixed_hand.txt);
* closed forms that need no rounding (impulse, constant);
* the constant table against its definition;
* the rounding: the integer result's deviation from the exact DFT has the
  size that independent uniform rounding errors of 1/2 after each product
  give (the same code in FP64 with injected noise), and does not grow with the
  input scale (so it is rounding, not a wrong formula);
* wrap-around: inputs are taken modulo 2^32, and without products (N <= 4)
  the transform is linear modulo 2^32;
* planted mistakes (a constant off by one, truncating instead of rounding)
  fail these pins.
"""
import math
import os

import numpy as np
import pytest

from oracle import build as OB
from oracle import direct as D
from oracle import qft as Q
from oracle import qft_fixed as F

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fixed_hand.txt")


def _pairs(s):
    return np.array([[int(v) for v in p.split(",")] for p in s.split(";")], dtype=np.int64)


def _hand_rows():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if line and not line.startswith("#"):
            n, xs, Xs = (t.strip() for t in line.split("|"))
            rows.append((int(n), _pairs(xs), _pairs(Xs)))
    return rows


def _c(a):
    return a[..., 0] + 1j * a[..., 1]


@pytest.mark.parametrize("r", range(1, 13))
def test_structure_equals_fp64_oracle(r):
    rng = np.random.default_rng(100 + r)
    N = 1 << r
    x = rng.standard_normal((3, N)) + 1j * rng.standard_normal((3, N))
    assert D.relative_l2(F.cdft_model(x), Q.qft(x)).max() < 1e-13


@pytest.mark.parametrize("row", _hand_rows())
def test_hand_values(row):
    N, x, X = row
    assert x.shape == (N, 2)
    assert np.array_equal(F.cdft_fixed(x[None])[0], X)


@pytest.mark.parametrize("r", [1, 2, 3, 5, 9, 12])
def test_impulse_and_constant_are_exact(r):
    N = 1 << r
    x = np.zeros((1, N, 2), np.int64)
    x[0, 0] = (12345, -77)               # impulse at 0: every bin equals x(0)
    X = F.cdft_fixed(x)
    assert (X[0, :, 0] == 12345).all() and (X[0, :, 1] == -77).all()
    x = np.zeros((1, N, 2), np.int64)
    x[0, :] = (3, -5)                    # constant: N x at k = 0, zero elsewhere
    X = F.cdft_fixed(x)
    assert tuple(X[0, 0]) == (3 * N, -5 * N) and (X[0, 1:] == 0).all()


def test_table_matches_definition():
    H, sh = F.secant_table_q(16)
    L = 1
    while 2 * L <= H.size:
        s = int(sh[L])
        hmax = 1 / (2 * math.cos(math.pi * (2 * L - 1) / (4 * L)))
        assert 2 ** (29 - s) <= hmax < 2 ** (30 - s)          # block exponent
        assert H[2 * L - 1] < 2 ** 30 and H[2 * L - 1] >= 2 ** 28
        m = np.arange(L)
        exact = 1 / (2 * np.cos(np.pi * (2 * m + 1) / (4 * L)))
        assert np.all(np.abs(H[L:2 * L] / 2.0 ** s - exact) <= 2.0 ** -(s + 1) * 1.0001)
        L *= 2
    assert H[1] == 759250125 and sh[1] == 30               # cos(pi/4) at s = 30


def _errors(r, scale, batch, seed):
    rng = np.random.default_rng(seed)
    N = 1 << r
    x = rng.integers(-scale, scale, (batch, N, 2))
    exact = OB.cdft(_c(x).astype(np.complex128))
    e_int = _c(F.cdft_fixed(x)) - exact
    e_mod = F.cdft_model(_c(x).astype(np.complex128), np.random.default_rng(seed + 1)) - exact
    return e_int, e_mod


@pytest.mark.parametrize("r", [6, 10, 13])
def test_rounding_matches_the_noise_model(r):
    """The integer deviation from the exact DFT against FP64 runs with an
    independent uniform error in [-1/2, 1/2) after every product: the RMS
    agree within a factor 2 and no bin exceeds c(n) times the model's RMS
    (c(n) = 2 sqrt(ln n + ln 1e9), as in tests/parity.py)."""
    N = 1 << r
    e_int, e_mod = _errors(r, 1 << (28 - r), 8, 40 + r)
    ri = np.sqrt(np.mean(np.abs(e_int) ** 2))
    rm = np.sqrt(np.mean(np.abs(e_mod) ** 2))
    assert 0.5 * rm <= ri <= 2.0 * rm, (ri, rm)
    c = 2 * math.sqrt(math.log(e_int.size) + math.log(1e9))
    assert np.abs(e_int).max() <= c * rm


def test_rounding_error_does_not_scale_with_the_input():
    """Absolute error of about the same size at input scales 2^8 and 2^16 at
    N = 2^10: it is the rounding of the products, not a wrong formula (which
    would scale with the input)."""
    r = 10
    a, _ = _errors(r, 1 << 8, 8, 7)
    b, _ = _errors(r, 1 << 16, 8, 7)
    ra, rb = np.sqrt(np.mean(np.abs(a) ** 2)), np.sqrt(np.mean(np.abs(b) ** 2))
    assert rb < 4 * ra and ra < 4 * rb, (ra, rb)


def test_wraparound():
    rng = np.random.default_rng(9)
    x = rng.integers(-(1 << 31), 1 << 31, (4, 64, 2))
    shifted = x + (rng.integers(-3, 4, x.shape) << 32)
    assert np.array_equal(F.cdft_fixed(x), F.cdft_fixed(shifted))
    a = rng.integers(-(1 << 31), 1 << 31, (4, 4, 2))
    b = rng.integers(-(1 << 31), 1 << 31, (4, 4, 2))
    wrap = lambda v: ((v + (1 << 31)) % (1 << 32)) - (1 << 31)  # noqa: E731
    assert np.array_equal(F.cdft_fixed(a + b), wrap(F.cdft_fixed(a) + F.cdft_fixed(b)))


def test_planted_mistakes_fail(monkeypatch):
    row = _hand_rows()[1]                       # N = 8, 1060.66 rounds to 1061
    orig = F._slice
    with monkeypatch.context() as m:           # truncation instead of rounding
        m.setattr(F._Int, "mul", lambda self, w, L: self.wrap(
            (w * orig(L)[1]) >> orig(L)[2]))
        assert not np.array_equal(F.cdft_fixed(row[1][None])[0], row[2])
    with monkeypatch.context() as m:           # one constant of slice 64 off by one
        def bad(L):
            h, H, s = orig(L)
            if L == 64:
                H = H.copy()
                H[5] += 1 << 8
            return h, H, s
        m.setattr(F, "_slice", bad)
        e_int, e_mod = _errors(10, 1 << 18, 4, 3)
        ri = np.sqrt(np.mean(np.abs(e_int) ** 2))
        rm = np.sqrt(np.mean(np.abs(e_mod) ** 2))
        assert ri > 2.0 * rm
