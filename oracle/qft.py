"""Oracle B: the improved QFT recursion, FP64, numpy.

Test infrastructure only (see ``oracle/__init__``).

This follows Pasquini, "Improved QFT algorithm for power-of-two FFT":

* the transforms of Sec. 2.1: DFT (eq. qft_0A), DCT-0 (eq. qft_0B), DST-0
  (eq. qft_0C), theta = 2*pi/N where N is the *periodization of the current
  call* (eq. qft_0D);
* the signal types of Table 1 (``tab:notation``): every function takes the
  stored time samples (``sto_n``, increasing n) and returns the stored
  frequency samples (``sto_k``, increasing k);
* the basic elaborations of Sec. 3 (even/odd time split, Sec. 3.1, eqs.
  qft_5A-5D and qft_6; even/odd harmonic split, Sec. 3.2, eqs. qft_1, qft_2,
  qft_4B; even-harmonic halving, Sec. 3.3, eqs. qft_9/qft_10; even-time
  halving, Sec. 3.4, eqs. qft_12/qft_13);
* the eight functions of Sec. 5.2: ``cdft`` and ``rdft`` (identical to the
  classical ones of Sec. 4.1/4.2), ``dct``, ``dct_ot``, ``dct_oo`` and their
  DST analogues (Sec. 5.2.4).

Every function works on arrays whose LAST axis holds the stored samples, so a
whole batch goes through one recursion. Arithmetic is IEEE FP64 (numpy never
fuses a multiply with an add).

Readings of the paper where it is silent or garbled (each one is also listed
with its justification in the design notes of the repository):

* eq. qft_38B: the printed right-hand side DCT[s_dc_oe](N/4) is identically
  zero for odd-n signals; the relation that holds is the two-term rule of eq.
  qft_38C at k = N/4-1 with the vanishing term DCT[s_dc_oe](N/4) dropped,
  i.e. DCT[s_dc_oo](N/4-1) = DCT[s_dc_oe](N/4-2).
* eq. qft_38C then applies for odd k <= N/4-3.
* ``dst_oo``: the special case sits at k = 1 (Sec. 5.2.4): DST[s_ds_oe](0) is
  zero, so DST[s_ds_oo](1) = DST[s_ds_oe](2); every other odd k, k = N/4-1
  included, takes the two-term sum.
* eq. qft_38A lists n in {0..N/4-1}; only odd n are stored in s_dc_oo, so the
  secant multiply runs over odd n only and never meets n = 0.
* the ``dct`` text names the even-time child s_ds_et; it is s_dc_et.
* the secant constant of the conversions is 1/(2 cos(theta n)) (eq. qft_26,
  eq. qft_38A); the "csc" of Sec. 4.7 is read as this secant.
* base cases: ``dct`` N=2, ``dst`` N=4, ``dct_ot``/``dst_ot`` N=4,
  ``dct_oo``/``dst_oo`` N=8 by the definitions (Sec. 5.2); the ``dst_ot`` base
  (one sample, sin(pi/2) = 1) is the identity; ``dst_oo`` N=8 is one multiply by
  sin(pi/4) (Sec. 6.1 counts cos(2*pi/8) as the one extra constant).
* ``cdft``/``rdft`` require N >= 2.

Operation counting (``Ops``): every real addition/subtraction and every real
multiplication is counted once per transform (the batch axes are not
counted). Sign changes and index relabelling are free; this is the model in
which Table 2 (``tab:costo_improved_qft``) states the cost.
"""
import numpy as np

__all__ = [
    "Ops", "SIGNAL_TYPES", "ln", "lk",
    "cdft", "rdft", "dct", "dst", "dct_ot", "dst_ot", "dct_oo", "dst_oo",
    "qft", "qft_adjoint",
]


class Ops:
    """Real-operation counter for ONE transform (batch axes not counted)."""

    def __init__(self):
        self.add = 0
        self.mul = 0

    @property
    def flop(self):
        return self.add + self.mul


# --------------------------------------------------------------------------
# Table 1 (tab:notation): storage sizes of the signal types used by the
# improved QFT, as functions of the periodization N.  ln = stored time cells,
# lk = stored frequency cells (eqs. qft_1A, qft_1B).
# --------------------------------------------------------------------------
SIGNAL_TYPES = {
    #           ln(N)                 lk(N)
    "cx_tt": (lambda N: 2 * N,        lambda N: 2 * N),
    "re_tt": (lambda N: N,            lambda N: N),
    "dc_tt": (lambda N: N // 2 + 1,   lambda N: N // 2 + 1),
    "dc_et": (lambda N: N // 4 + 1,   lambda N: N // 4 + 1),
    "dc_ot": (lambda N: N // 4,       lambda N: N // 4),
    "dc_oe": (lambda N: N // 8,       lambda N: N // 8),
    "dc_oo": (lambda N: N // 8,       lambda N: N // 8),
    "ds_tt": (lambda N: N // 2 - 1,   lambda N: N // 2 - 1),
    "ds_et": (lambda N: N // 4 - 1,   lambda N: N // 4 - 1),
    "ds_ot": (lambda N: N // 4,       lambda N: N // 4),
    "ds_oe": (lambda N: N // 8,       lambda N: N // 8),
    "ds_oo": (lambda N: N // 8,       lambda N: N // 8),
}


def ln(sig_type, N):
    return SIGNAL_TYPES[sig_type][0](N)


def lk(sig_type, N):
    return SIGNAL_TYPES[sig_type][1](N)


def _check_in(x, sig_type, N):
    if x.shape[-1] != ln(sig_type, N):
        raise AssertionError(
            f"{sig_type}(N={N}): {x.shape[-1]} time cells, Table 1 says {ln(sig_type, N)}")


def _check_out(X, sig_type, N):
    if X.shape[-1] != lk(sig_type, N):
        raise AssertionError(
            f"{sig_type}(N={N}): {X.shape[-1]} frequency cells, Table 1 says {lk(sig_type, N)}")


def _conserved(parent, N, children):
    """Sec. 6.1 (eqs. qft_42/qft_43 and 'similar relations hold for any other
    function'): the children of every improved-QFT function hold exactly the
    parent's ln and lk in total."""
    tot_ln = sum(ln(t, n) for t, n in children)
    tot_lk = sum(lk(t, n) for t, n in children)
    if tot_ln != ln(parent, N) or tot_lk != lk(parent, N):
        raise AssertionError(f"ln/lk not conserved in {parent}(N={N}): {children}")


def _secant(n, N):
    """1/(2 cos(theta*n)), theta = 2*pi/N (eqs. qft_26, qft_38A), FP64."""
    return 1.0 / (2.0 * np.cos(2.0 * np.pi * n / N))


# --------------------------------------------------------------------------
# The DCT family (Sec. 5.2.1 - 5.2.3)
# --------------------------------------------------------------------------
def dct(s, N, ops):
    """``dct``: s_dc_tt, time n = 0..N/2 -> DCT-0 (eq. qft_0B), k = 0..N/2."""
    _check_in(s, "dc_tt", N)
    if N == 2:
        # definition: S(k) = s(0) + s(1) cos(pi k)
        S = np.stack([s[..., 0] + s[..., 1], s[..., 0] - s[..., 1]], axis=-1)
        ops.add += 2
        _check_out(S, "dc_tt", N)
        return S
    # forward: separation of even and odd time indices (Sec. 3.1, eqs. 5A/5B)
    s_et = s[..., 0::2]             # n = 0, 2, ..., N/2      (s_dc_et)
    s_ot = s[..., 1::2]             # n = 1, 3, ..., N/2 - 1  (s_dc_ot)
    _conserved("dc_tt", N, [("dc_et", N), ("dc_ot", N)])
    # even time indices halving (Sec. 3.4, eq. 12): s_A(n_A) = s_et(2 n_A),
    # periodization N/2, type s_dc_tt; its DCT equals DCT[s_et] (eq. 13).
    E = dct(s_et, N // 2, ops)      # k = 0..N/4
    O = dct_ot(s_ot, N, ops)        # k = 0..N/4-1
    # backward (eqs. 5C, 5D, 6)
    q = N // 4
    S = np.empty(s.shape[:-1] + (N // 2 + 1,), dtype=s.dtype)
    S[..., 0:q] = E[..., 0:q] + O                     # S(k),      k < N/4
    S[..., N // 2:q:-1] = E[..., 0:q] - O             # S(N/2-k),  k < N/4
    S[..., q] = E[..., q]                             # S(N/4)
    ops.add += 2 * q
    _check_out(S, "dc_tt", N)
    return S


def dct_ot(s, N, ops):
    """``dct_ot``: s_dc_ot, time n = 1,3,..,N/2-1 -> k = 0..N/4-1."""
    _check_in(s, "dc_ot", N)
    if N == 4:
        # definition: one sample n = 1, one harmonic k = 0: cos(0) = 1
        S = s.copy()
        _check_out(S, "dc_ot", N)
        return S
    # forward: separation of even and odd harmonics (Sec. 3.2, eqs. qft_1, qft_2).
    # Stored sample j holds n = 2j+1; its mirror N/2 - n holds index N/4-1-j.
    m = N // 8                      # samples with n in [0, N/4-1]: j < N/8
    a = s[..., :m]
    b = s[..., ::-1][..., :m]       # s(N/2 - n)
    s_oe = a + b                    # even harmonics child, s_dc_oe
    s_oo = a - b                    # odd harmonics child,  s_dc_oo
    ops.add += 2 * m
    _conserved("dc_ot", N, [("dc_oe", N), ("dc_oo", N)])
    # even harmonics halving (Sec. 3.3, eqs. 9/10): s_dc_oe of periodization N
    # is s_A_dc_ot of periodization N/2, DCT[s_oe](2 k_A) = DCT[s_A](k_A).
    A = dct_ot(s_oe, N // 2, ops)   # k_A = 0..N/8-1  -> even k = 2 k_A
    B = dct_oo(s_oo, N, ops)        # odd k = 1, 3, .., N/4-1
    # backward: interleave (eq. qft_4B)
    S = np.empty(s.shape[:-1] + (N // 4,), dtype=s.dtype)
    S[..., 0::2] = A
    S[..., 1::2] = B
    _check_out(S, "dc_ot", N)
    return S


def dct_oo(s, N, ops):
    """``dct_oo``: s_dc_oo, time n = 1,3,..,N/4-1 -> odd k = 1,3,..,N/4-1."""
    _check_in(s, "dc_oo", N)
    if N == 8:
        # definition: n = 1, k = 1: cos(2*pi/8)
        S = s * np.cos(2.0 * np.pi / 8.0)
        ops.mul += 1
        _check_out(S, "dc_oo", N)
        return S
    # forward: eq. qft_38A on the stored (odd) n only
    n = 2 * np.arange(N // 8) + 1
    s_oe = s * _secant(n, N)        # s_dc_oe, periodization N
    ops.mul += N // 8
    # even harmonics halving (Sec. 3.3): s_A_dc_ot of periodization N/2, which
    # is processed exactly as ``dct_ot`` processes s_dc_ot (Sec. 5.2.3).
    _conserved("dc_oo", N, [("dc_ot", N // 2)])
    T = dct_ot(s_oe, N // 2, ops)   # T(j) = DCT[s_oe](2j), j = 0..N/8-1
    # backward: eq. qft_38C for odd k = 2j+1 <= N/4-3, and the corrected
    # eq. qft_38B at k = N/4-1 (DCT[s_oe](N/4) = 0).
    S = np.empty_like(T)
    S[..., :-1] = T[..., :-1] + T[..., 1:]
    S[..., -1] = T[..., -1]
    ops.add += N // 8 - 1
    _check_out(S, "dc_oo", N)
    return S


# --------------------------------------------------------------------------
# The DST family (Sec. 5.2.4): same chains with dc -> ds, plus the two
# differences the paper lists (dst base at N = 4, dst_oo special case at k = 1).
# --------------------------------------------------------------------------
def dst(s, N, ops):
    """``dst``: s_ds_tt, time n = 1..N/2-1 -> DST-0 (eq. qft_0C), k = 1..N/2-1."""
    _check_in(s, "ds_tt", N)
    if N == 4:
        # definition: n = 1, k = 1: sin(pi/2) = 1
        S = s.copy()
        _check_out(S, "ds_tt", N)
        return S
    # forward: separation of even and odd time indices (Sec. 3.1).  The stored
    # index j holds n = j + 1.
    s_et = s[..., 1::2]             # n = 2, 4, .., N/2-2   (s_ds_et)
    s_ot = s[..., 0::2]             # n = 1, 3, .., N/2-1   (s_ds_ot)
    _conserved("ds_tt", N, [("ds_et", N), ("ds_ot", N)])
    # even time halving (Sec. 3.4): s_A_ds_tt, periodization N/2, n_A = 1..N/4-1
    E = dst(s_et, N // 2, ops)      # k = 1..N/4-1
    O = dst_ot(s_ot, N, ops)        # k = 1..N/4
    # backward: eqs. 5C, 5D, 6 with the roles of the even and odd children
    # swapped (Sec. 3.1, DST case).  Stored index j <-> k = j + 1.
    q = N // 4
    S = np.empty(s.shape[:-1] + (N // 2 - 1,), dtype=s.dtype)
    # k = 1..N/4-1
    S[..., 0:q - 1] = O[..., 0:q - 1] + E                 # S(k)
    # S(N/2 - k) for k = 1..N/4-1 -> stored index N/2-k-1 = N/2-2 .. N/4
    S[..., N // 2 - 2:q - 1:-1] = O[..., 0:q - 1] - E
    S[..., q - 1] = O[..., q - 1]                         # S(N/4)
    ops.add += 2 * (q - 1)
    _check_out(S, "ds_tt", N)
    return S


def dst_ot(s, N, ops):
    """``dst_ot``: s_ds_ot, time n = 1,3,..,N/2-1 -> k = 1..N/4."""
    _check_in(s, "ds_ot", N)
    if N == 4:
        S = s.copy()                # n = 1, k = 1: sin(pi/2) = 1
        _check_out(S, "ds_ot", N)
        return S
    # forward: harmonic separation with the DST role swap (Sec. 3.2): the
    # even-harmonics child takes the difference, the odd one the sum.
    m = N // 8
    a = s[..., :m]
    b = s[..., ::-1][..., :m]       # s(N/2 - n)
    s_oe = a - b                    # s_ds_oe (even k)
    s_oo = a + b                    # s_ds_oo (odd k)
    ops.add += 2 * m
    _conserved("ds_ot", N, [("ds_oe", N), ("ds_oo", N)])
    A = dst_ot(s_oe, N // 2, ops)   # k_A = 1..N/8 -> even k = 2 k_A
    B = dst_oo(s_oo, N, ops)        # odd k = 1..N/4-1
    # backward: interleave (eq. qft_4B).  Stored index j <-> k = j + 1.
    S = np.empty(s.shape[:-1] + (N // 4,), dtype=s.dtype)
    S[..., 1::2] = A                # k = 2, 4, .., N/4
    S[..., 0::2] = B                # k = 1, 3, .., N/4-1
    _check_out(S, "ds_ot", N)
    return S


def dst_oo(s, N, ops):
    """``dst_oo``: s_ds_oo, time n = 1,3,..,N/4-1 -> odd k = 1,3,..,N/4-1."""
    _check_in(s, "ds_oo", N)
    if N == 8:
        S = s * np.sin(2.0 * np.pi / 8.0)   # n = 1, k = 1
        ops.mul += 1
        _check_out(S, "ds_oo", N)
        return S
    n = 2 * np.arange(N // 8) + 1
    s_oe = s * _secant(n, N)        # same conversion as eq. qft_38A
    ops.mul += N // 8
    _conserved("ds_oo", N, [("ds_ot", N // 2)])
    T = dst_ot(s_oe, N // 2, ops)   # T(j) = DST[s_oe](2(j+1)), j = 0..N/8-1
    # backward: DST[s_oo](k) = DST[s_oe](k-1) + DST[s_oe](k+1), odd k, with the
    # special case k = 1 where DST[s_oe](0) = 0.
    S = np.empty_like(T)
    S[..., 0] = T[..., 0]
    S[..., 1:] = T[..., :-1] + T[..., 1:]
    ops.add += N // 8 - 1
    _check_out(S, "ds_oo", N)
    return S


# --------------------------------------------------------------------------
# rdft and cdft (Sec. 4.1, 4.2; identical in the improved QFT, Sec. 5.2)
# --------------------------------------------------------------------------
def rdft(s, N, ops):
    """``rdft``: s_re_tt (real, n = 0..N-1) -> (Re S(k), k = 0..N/2;
    Im S(k), k = 1..N/2-1)."""
    _check_in(s, "re_tt", N)
    if N == 2:
        re = np.stack([s[..., 0] + s[..., 1], s[..., 0] - s[..., 1]], axis=-1)
        ops.add += 2
        return re, s[..., :0]
    h = N // 2
    fwd = s[..., 1:h]               # s(n),   n = 1..N/2-1
    rev = s[..., :h:-1]             # s(N-n), n = 1..N/2-1
    c = np.empty(s.shape[:-1] + (h + 1,), dtype=s.dtype)
    c[..., 0] = s[..., 0]
    c[..., h] = s[..., h]
    c[..., 1:h] = fwd + rev         # s_dc_tt
    d = fwd - rev                   # s_ds_tt
    ops.add += 2 * (h - 1)
    _conserved("re_tt", N, [("dc_tt", N), ("ds_tt", N)])
    C = dct(c, N, ops)              # Re RDFT(k) = DCT(k),  k = 0..N/2
    D = dst(d, N, ops)              # Im RDFT(k) = -DST(k), k = 1..N/2-1
    return C, -D


def cdft(z, N, ops):
    """``cdft``: s_cx_tt (complex, n = 0..N-1) -> S(k), k = 0..N-1."""
    z = np.asarray(z)
    if z.shape[-1] != N:
        raise AssertionError("cdft: length mismatch")
    if N == 2:
        S = np.stack([z[..., 0] + z[..., 1], z[..., 0] - z[..., 1]], axis=-1)
        ops.add += 4
        return S
    # children: real and imaginary parts (Sec. 4.1)
    re1, im1 = rdft(np.ascontiguousarray(z.real), N, ops)
    re2, im2 = rdft(np.ascontiguousarray(z.imag), N, ops)
    h = N // 2
    S = np.empty(z.shape, dtype=np.complex128)
    S[..., 0] = re1[..., 0] + 1j * re2[..., 0]
    S[..., h] = re1[..., h] + 1j * re2[..., h]
    r1, r2 = re1[..., 1:h], re2[..., 1:h]
    S[..., 1:h].real = r1 - im2                   # Re S(k)
    S[..., 1:h].imag = im1 + r2                   # Im S(k)
    S[..., N - 1:h:-1].real = r1 + im2            # Re S(N-k)
    S[..., N - 1:h:-1].imag = r2 - im1            # Im S(N-k)
    ops.add += 4 * (h - 1)
    return S


def qft(x, ops=None):
    """Forward unnormalised CDFT of the last axis by the improved QFT."""
    x = np.asarray(x, dtype=np.complex128)
    N = x.shape[-1]
    if N < 2 or (N & (N - 1)):
        raise ValueError("N must be a power of two >= 2")
    return cdft(x, N, ops if ops is not None else Ops())


def qft_adjoint(X, ops=None):
    """Conjugate-transpose map F^H X = conj(F conj(X)), evaluated through the
    same forward recursion (no new arithmetic: conjugation is a sign change)."""
    X = np.asarray(X, dtype=np.complex128)
    return np.conj(qft(np.conj(X), ops))

