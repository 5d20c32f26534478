"""Pins for Oracle B (the improved-QFT recursion in FP64, Secs. 3-5).

What pins it, other than itself:
  * Oracle A (the DFT definition, itself pinned by hand values and closed
    forms) for r = 1..12;
  * every one of the eight functions against the definition of its transform
    (eqs. qft_0B / qft_0C) evaluated by brute force over the index sets of
    Table 1;
  * the derived equivalences with library transforms (scipy DCT/DST types 2
    and 4, halved) for the dct_ot/dct_oo/dst_ot/dst_oo signals;
  * the operation counters against the closed forms of Table 2 and the
    printed rows of Tables 3-5;
  * planted mistakes in the oracle (a dropped term, a swapped sign, the
    literal printed form of eq. qft_38B) must break one of these pins.
The C copy (oracle/qft_ref.c, the timed CPU baseline) is pinned the same way.
"""
import os
from fractions import Fraction as F

import numpy as np
import pytest
import scipy.fft as sfft

from oracle import direct as D
from oracle import qft as Q

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-0.5, 0.5, shape) + 1j * rng.uniform(-0.5, 0.5, shape)


@pytest.mark.parametrize("r", range(1, 13))
def test_qft_equals_dft(r):
    N = 1 << r
    x = _rand((3, N), r)
    err = D.relative_l2(Q.qft(x), D.dft(x)).max()
    assert err < 1e-13


def test_adjoint_equals_dft_adjoint():
    x = _rand((2, 128), 3)
    np.testing.assert_allclose(Q.qft_adjoint(x), D.dft_adjoint(x), atol=1e-12)


# --- each function against the definition of its transform -----------------
def _dct_def(vals, ns, ks, N):
    th = 2 * np.pi / N
    return np.array([sum(v * np.cos(th * n * k) for v, n in zip(vals, ns)) for k in ks])


def _dst_def(vals, ns, ks, N):
    th = 2 * np.pi / N
    return np.array([sum(v * np.sin(th * n * k) for v, n in zip(vals, ns)) for k in ks])


# (function, definition, sto_n(N), sto_k(N), smallest N) from Table 1
CASES = [
    (Q.dct, _dct_def, lambda N: range(0, N // 2 + 1), lambda N: range(0, N // 2 + 1), 2),
    (Q.dst, _dst_def, lambda N: range(1, N // 2), lambda N: range(1, N // 2), 4),
    (Q.dct_ot, _dct_def, lambda N: range(1, N // 2, 2), lambda N: range(0, N // 4), 4),
    (Q.dst_ot, _dst_def, lambda N: range(1, N // 2, 2), lambda N: range(1, N // 4 + 1), 4),
    (Q.dct_oo, _dct_def, lambda N: range(1, N // 4, 2), lambda N: range(1, N // 4, 2), 8),
    (Q.dst_oo, _dst_def, lambda N: range(1, N // 4, 2), lambda N: range(1, N // 4, 2), 8),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0].__name__)
@pytest.mark.parametrize("r", range(1, 8))
def test_function_matches_definition(case, r):
    fn, defn, ston, stok, nmin = case
    N = 1 << r
    if N < nmin:
        pytest.skip("below the function's base case")
    ns, ks = list(ston(N)), list(stok(N))
    vals = np.random.default_rng(r).standard_normal(len(ns))
    got = fn(vals, N, Q.Ops())
    np.testing.assert_allclose(got, defn(vals, ns, ks, N), atol=1e-12)


@pytest.mark.parametrize("r", range(3, 12))
def test_ot_oo_are_dct_dst_types_2_and_4(r):
    """Derived identity: s_dc_ot (periodization N) is a DCT-II of length
    M = N/4 and s_dc_oo a DCT-IV of length N/8 (likewise DST); scipy's
    unnormalised types 2 and 4 carry a factor 2."""
    N = 1 << r
    rng = np.random.default_rng(100 + r)
    y = rng.standard_normal(N // 4)
    np.testing.assert_allclose(Q.dct_ot(y, N, Q.Ops()), sfft.dct(y, 2) / 2, atol=1e-11)
    np.testing.assert_allclose(Q.dst_ot(y, N, Q.Ops()), sfft.dst(y, 2) / 2, atol=1e-11)
    w = rng.standard_normal(N // 8)
    np.testing.assert_allclose(Q.dct_oo(w, N, Q.Ops()), sfft.dct(w, 4) / 2, atol=1e-11)
    np.testing.assert_allclose(Q.dst_oo(w, N, Q.Ops()), sfft.dst(w, 4) / 2, atol=1e-11)


# --- operation counts --------------------------------------------------------
def _table2(N):
    """Table 2 (tab:costo_improved_qft) closed forms, log = log2."""
    r = N.bit_length() - 1
    NL = N * r
    return {
        "CDFT": (NL - 3 * N + 4, 3 * NL - 3 * N + 4),
        "RDFT": (F(NL, 2) - F(3 * N, 2) + 2, F(3 * NL, 2) - F(5 * N, 2) + 4),
        "DCT-0": (F(NL, 4) - F(3 * N, 4) + 1, F(3 * NL, 4) - F(7 * N, 4) + r + 3),
        "DST-0": (F(NL, 4) - F(3 * N, 4) + 1, F(3 * NL, 4) - F(7 * N, 4) - r + 3),
    }


def _count(kind, N):
    ops = Q.Ops()
    if kind == "CDFT":
        Q.cdft(np.zeros(N, complex), N, ops)
    elif kind == "RDFT":
        Q.rdft(np.zeros(N), N, ops)
    elif kind == "DCT-0":
        Q.dct(np.zeros(N // 2 + 1), N, ops)
    else:
        Q.dst(np.zeros(N // 2 - 1), N, ops)
    return ops.mul, ops.add


@pytest.mark.parametrize("kind,rmin", [("CDFT", 2), ("RDFT", 2), ("DCT-0", 2), ("DST-0", 3)])
@pytest.mark.parametrize("r", range(2, 17))
def test_op_counts_match_table2(kind, rmin, r):
    if r < rmin:
        pytest.skip("closed form starts at a larger N")
    N = 1 << r
    mul, add = _count(kind, N)
    emul, eadd = _table2(N)[kind]
    assert (mul, add) == (emul, eadd)


def _tables_3_5():
    rows = []
    with open(os.path.join(GOLD, "table2_to_5.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(tuple(int(v) for v in line.split()))
    return rows


@pytest.mark.parametrize("row", _tables_3_5(), ids=lambda r: f"N{r[0]}")
def test_op_counts_match_tables_3_to_5(row):
    N, adds, muls, flops, printed = row
    mul, add = _count("CDFT", N)
    assert (add, mul, add + mul) == (adds, muls, flops)
    if printed != adds:
        assert N == 512 and printed == 12290  # the one misprint


def test_constant_set():
    """Sec. 6.1: the only constants are the secants 1/(2 cos(theta n)) and
    cos(2 pi / 8).  Expressed at the root periodization N, the secants used are
    those of q = 1..N/4-1 except q = N/8, whose value 1/(2 cos(pi/4)) equals
    the base-case constant cos(2 pi / 8): N/4 - 1 distinct values in all."""
    N = 1 << 10
    seen = set()
    orig_sec = Q._secant

    def rec_sec(n, NN):
        for nn in np.atleast_1d(n):
            seen.add(int(nn) * (N // NN))  # index at the root periodization
        return orig_sec(n, NN)

    Q._secant = rec_sec
    try:
        Q.qft(np.zeros(N, complex))
    finally:
        Q._secant = orig_sec
    assert seen == set(range(1, N // 4)) - {N // 8}
    # equal as real numbers; one FP64 ulp apart after rounding, equal in FP32
    assert abs(orig_sec(1, 8) - np.cos(2 * np.pi / 8)) <= 2.3e-16
    assert np.float32(orig_sec(1, 8)) == np.float32(np.cos(2 * np.pi / 8))


# --- storage sizes (Table 1) ------------------------------------------------
def test_storage_size_checks_fire():
    with pytest.raises(AssertionError):
        Q.dct(np.zeros(7), 16, Q.Ops())  # dc_tt at N=16 stores 9 samples
    with pytest.raises(AssertionError):
        Q.dst_oo(np.zeros(3), 32, Q.Ops())  # ds_oo at N=32 stores 4


def test_conservation_check_fires():
    """The Sec. 6.1 ln/lk conservation check rejects a child list that does
    not hold exactly the parent's cells (eqs. qft_42/qft_43), and accepts the
    ones the recursion uses."""
    Q._conserved("dc_ot", 32, [("dc_oe", 32), ("dc_oo", 32)])
    Q._conserved("dc_tt", 32, [("dc_et", 32), ("dc_ot", 32)])
    with pytest.raises(AssertionError):  # one child missing
        Q._conserved("dc_ot", 32, [("dc_oe", 32)])
    with pytest.raises(AssertionError):  # a child at the wrong periodization
        Q._conserved("dc_oo", 32, [("dc_ot", 32)])
    with pytest.raises(AssertionError):  # the DST child list of a DCT parent
        Q._conserved("dc_tt", 32, [("ds_et", 32), ("ds_ot", 32)])


def test_table1_sizes():
    # a few rows of Table 1 transcribed as numbers (N = 64)
    N = 64
    assert (Q.ln("dc_tt", N), Q.ln("dc_et", N), Q.ln("dc_ot", N)) == (33, 17, 16)
    assert (Q.ln("ds_tt", N), Q.ln("ds_et", N), Q.ln("ds_ot", N)) == (31, 15, 16)
    assert (Q.ln("dc_oo", N), Q.lk("ds_oe", N), Q.lk("re_tt", N)) == (8, 8, 64)


# --- planted mistakes must be caught -----------------------------------------
def _pins_pass():
    x = _rand((1, 64), 9)
    return D.relative_l2(Q.qft(x), D.dft(x)).max() < 1e-12


def test_pins_catch_planted_mistakes(monkeypatch):
    assert _pins_pass()

    def bad_secant(n, N):  # wrong constant: 1/cos instead of 1/(2cos)
        return 1.0 / np.cos(2.0 * np.pi * n / N)

    with monkeypatch.context() as m:
        m.setattr(Q, "_secant", bad_secant)
        assert not _pins_pass()

    orig_dst_oo = Q.dst_oo

    def dst_oo_dropped_term(s, N, ops):  # special case at k = N/4-1 instead of k = 1
        if N == 8:
            return orig_dst_oo(s, N, ops)
        n = 2 * np.arange(N // 8) + 1
        T = Q.dst_ot(s * Q._secant(n, N), N // 2, ops)
        S = np.empty_like(T)
        S[..., :-1] = T[..., :-1] + T[..., 1:]
        S[..., -1] = T[..., -1]
        return S

    with monkeypatch.context() as m:
        m.setattr(Q, "dst_oo", dst_oo_dropped_term)
        assert not _pins_pass()


def test_literal_eq38B_is_wrong():
    """The printed eq. qft_38B, DCT[s_dc_oo](N/4-1) = DCT[s_dc_oe](N/4), would
    set the last odd harmonic to DCT[s_dc_oe](N/4) = 0 (cos(pi n/2) = 0 for odd
    n); the corrected reading DCT[s_dc_oe](N/4-2) matches the definition."""
    N = 32
    rng = np.random.default_rng(2)
    s = rng.standard_normal(N // 8)
    ns = range(1, N // 4, 2)
    th = 2 * np.pi / N
    t = s * Q._secant(np.array(list(ns)), N)
    assert abs(sum(tv * np.cos(th * n * (N // 4)) for tv, n in zip(t, ns))) < 1e-12
    exact = _dct_def(s, ns, [N // 4 - 1], N)[0]
    corrected = sum(tv * np.cos(th * n * (N // 4 - 2)) for tv, n in zip(t, ns))
    assert abs(corrected - exact) < 1e-12
    assert abs(exact) > 1e-3  # so the literal value 0 is wrong
    got = Q.dct_oo(s, N, Q.Ops())[-1]
    assert abs(got - exact) < 1e-12


# --- the C copy used as the timed CPU baseline -------------------------------
@pytest.fixture(scope="module")
def cref():
    from oracle import build as OB
    return OB


@pytest.mark.parametrize("r", [1, 2, 3, 5, 8, 11, 12])
def test_c_oracle_equals_dft(cref, r):
    N = 1 << r
    x = _rand((2, N), 40 + r)
    assert D.relative_l2(cref.cdft(x), D.dft(x)).max() < 1e-13


def test_c_oracle_large_bins(cref):
    N = 1 << 16
    x = _rand((1, N), 77)
    X = cref.cdft(x)
    bins = np.array([0, 1, 2, 3, N // 4, N // 2 - 1, N // 2, N - 1, 12345, 54321])
    ref = D.dft_bins(x, bins)
    assert np.max(np.abs(X[:, bins] - ref)) / np.sqrt(np.mean(np.abs(ref) ** 2)) < 1e-12
    # Parseval over the whole transform
    np.testing.assert_allclose(np.sum(np.abs(X) ** 2), N * np.sum(np.abs(x) ** 2), rtol=1e-12)
