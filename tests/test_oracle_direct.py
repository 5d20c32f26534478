"""Pins for Oracle A (the O(N^2) DFT by its definition, Sec. 2.1 eq. qft_0A).

Each check comes from something other than the oracle itself: hand-worked
values, closed forms of special inputs, unitarity/Parseval, linearity, and the
library routine numpy.fft.fft as an independent special case.
"""
import os

import numpy as np
import pytest

from oracle import direct as D

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _parse_pairs(s):
    vals = []
    for p in s.split(";"):
        re_, im_ = p.split(",")
        vals.append(complex(float(re_), float(im_)))
    return np.array(vals)


def _hand_rows():
    rows = []
    with open(os.path.join(GOLD, "dft_hand.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            n, xs, Xs = (t.strip() for t in line.split("|"))
            rows.append((int(n), _parse_pairs(xs), _parse_pairs(Xs)))
    return rows


@pytest.mark.parametrize("row", _hand_rows())
def test_hand_values(row):
    N, x, X = row
    assert x.size == N
    np.testing.assert_allclose(D.dft(x[None])[0], X, atol=1e-15)


@pytest.mark.parametrize("N", [1, 2, 3, 8, 12, 64, 1000, 4096])
def test_unit_roots_exact_points(N):
    w = D.unit_roots(N)
    assert np.all(np.abs(np.abs(w) - 1.0) < 5e-16)
    assert w[0] == 1.0
    if N % 2 == 0:
        assert w[N // 2] == -1.0
    if N % 4 == 0:
        assert w[N // 4] == -1j and w[3 * N // 4] == 1j
    if N % 8 == 0:
        r = np.sqrt(0.5)
        assert abs(w[N // 8] - (r - 1j * r)) < 3e-16
    # conjugate symmetry w[N-m] = conj(w[m])
    m = np.arange(1, N)
    assert np.all(w[N - m] == np.conj(w[m]))


@pytest.mark.parametrize("N", [2, 8, 64, 256, 1024])
def test_impulse_gives_all_ones(N):
    x = np.zeros((1, N), complex)
    x[0, 0] = 1.0
    np.testing.assert_allclose(D.dft(x)[0], np.ones(N), atol=0)


@pytest.mark.parametrize("N,n0", [(8, 3), (64, 5), (256, 77), (1024, 513)])
def test_shifted_impulse(N, n0):
    x = np.zeros((1, N), complex)
    x[0, n0] = 1.0
    k = np.arange(N)
    closed = np.exp(-2j * np.pi * ((n0 * k) % N) / N)
    np.testing.assert_allclose(D.dft(x)[0], closed, atol=1e-14)


@pytest.mark.parametrize("N", [4, 32, 512])
def test_constant_gives_N_at_dc(N):
    c = 0.75 - 0.25j
    X = D.dft(np.full((1, N), c))[0]
    assert abs(X[0] - N * c) < 1e-12
    assert np.max(np.abs(X[1:])) < 1e-12 * N


@pytest.mark.parametrize("N,f", [(16, 3), (256, 200), (4096, 1234)])
def test_integer_tone_single_bin(N, f):
    n = np.arange(N)
    x = np.exp(2j * np.pi * ((f * n) % N) / N)[None]
    X = D.dft(x)[0]
    assert abs(X[f] - N) < 1e-9
    mask = np.ones(N, bool)
    mask[f] = False
    assert np.max(np.abs(X[mask])) < 1e-9


def test_parseval_and_linearity():
    rng = np.random.default_rng(11)
    N = 512
    x = rng.standard_normal((3, N)) + 1j * rng.standard_normal((3, N))
    y = rng.standard_normal((3, N)) + 1j * rng.standard_normal((3, N))
    X, Y = D.dft(x), D.dft(y)
    np.testing.assert_allclose(np.sum(np.abs(X) ** 2, -1), N * np.sum(np.abs(x) ** 2, -1),
                               rtol=1e-12)
    a, b = 0.3 - 1.1j, -2.0 + 0.5j
    np.testing.assert_allclose(D.dft(a * x + b * y), a * X + b * Y, atol=1e-10)


@pytest.mark.parametrize("N", [2, 16, 128, 1024, 4096])
def test_matches_numpy_fft(N):
    rng = np.random.default_rng(N)
    x = rng.uniform(-1, 1, (2, N)) + 1j * rng.uniform(-1, 1, (2, N))
    err = D.relative_l2(D.dft(x), np.fft.fft(x)).max()
    assert err < 1e-14


def test_bins_and_adjoint():
    rng = np.random.default_rng(5)
    N = 256
    x = rng.standard_normal((2, N)) + 1j * rng.standard_normal((2, N))
    bins = np.array([0, 1, 17, 128, 255])
    np.testing.assert_allclose(D.dft_bins(x, bins), D.dft(x)[:, bins], atol=1e-12)
    # F^H F = N I
    np.testing.assert_allclose(D.dft_adjoint(D.dft(x)), N * x, atol=1e-10)
    np.testing.assert_allclose(D.dft_adjoint(x), N * np.fft.ifft(x), atol=1e-11)


# --- the accuracy measures used by every parity test -------------------------
def test_relative_l2_hand_values():
    """eq. qft_44 before averaging: ||S - S_exact||_2 / ||S_exact||_2 per
    signal.  Hand values: a 10% scaling gives exactly 0.1; S_exact = (3, 4)
    (norm 5) with one component off by 1 gives 1/5 (0.04 if the square root
    were dropped); S = 2 S_exact gives 1 (0.5 if normalised by ||S||); S = 0
    gives 1; one value per signal along the chosen axis."""
    e = np.array([3.0 + 0j, 4.0])
    assert D.relative_l2(1.1 * e, e) == pytest.approx(0.1, rel=1e-15, abs=0)
    assert D.relative_l2(np.array([3.0, 5.0]), e) == pytest.approx(0.2, rel=1e-15)
    assert D.relative_l2(2 * e, e) == pytest.approx(1.0, rel=1e-15)
    assert D.relative_l2(np.zeros(2), e) == pytest.approx(1.0, rel=1e-15)
    # complex parts: S_exact = (1, i), S = (1 + i, i) -> |i| / sqrt(2)
    assert D.relative_l2(np.array([1 + 1j, 1j]), np.array([1, 1j])) == \
        pytest.approx(1 / np.sqrt(2), rel=1e-15)
    # per signal along the axis: rows (0.1, 1.0); along axis 0 (columns)
    Sx = np.stack([1.1 * e, 2 * e])
    Ex = np.stack([e, e])
    np.testing.assert_allclose(D.relative_l2(Sx, Ex), [0.1, 1.0], rtol=1e-15)
    np.testing.assert_allclose(D.relative_l2(Sx, Ex, axis=0),
                               [np.sqrt(0.1 ** 2 + 1) / np.sqrt(2)] * 2, rtol=1e-15)


def test_bin_errors_hand_values():
    """|S(k) - S_exact(k)| / rms(S_exact): S_exact = (3, 4i) has rms
    sqrt(12.5); an error of 1 in bin 1 gives (0, 1/sqrt(12.5)); relative_l2
    is the root mean square of the bin errors."""
    e = np.array([3.0 + 0j, 4.0j])
    got = D.bin_errors(np.array([3.0, 5.0j]), e)
    np.testing.assert_allclose(got, [0.0, 1 / np.sqrt(12.5)], rtol=1e-15)
    rng = np.random.default_rng(3)
    S = rng.standard_normal((4, 64)) + 1j * rng.standard_normal((4, 64))
    E = rng.standard_normal((4, 64)) + 1j * rng.standard_normal((4, 64))
    np.testing.assert_allclose(np.sqrt(np.mean(D.bin_errors(S, E) ** 2, -1)),
                               D.relative_l2(S, E), rtol=1e-13)
    assert D.bin_errors(S, E).shape == (4, 64)
