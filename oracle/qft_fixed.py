"""Oracle F: the improved QFT in fixed point (integers).

Test infrastructure only (see ``oracle/__init__``).

The paper recommends the improved QFT for fixed-point implementations, where
a multiplication costs more than an addition (Sec. 1 and Sec. 7).  This
module runs the eight functions of Sec. 5.2 (``cdft``, ``rdft``, ``dct``,
``dct_ot``, ``dct_oo`` and the DST analogues; Sec. 3 for the elaborations)
on integers, in the paper's order, with the readings of ``oracle/qft.py``.

Number format (the rule the GPU path implements too):

* every sample is a signed 32-bit integer; additions and subtractions wrap
  modulo 2^32 (two's complement), so every result is defined for any input;
* the only multiplications are the secant conversions (eq. qft_38A) and the
  N = 8 base cases.  The constants of periodization P = 8L, h_L(m) =
  1/(2 cos(pi (2m+1) / (4L))), m < L, are block scaled: one shift per slice,
  s_L = 30 - e_L with e_L the binary exponent of the slice's largest constant
  h_L(L-1) (frexp: h < 2^e_L), and mantissas H_L(m) = floor(h_L(m) 2^s_L + 1/2)
  < 2^30 (FP64, cosine from the C library, rounded once).  The base cases
  DCT-IV(1) = x cos(pi/4) and DST-IV(1) = x sin(pi/4) use the slice L = 1,
  whose one constant 1/(2 cos(pi/4)) equals cos(pi/4) = sin(pi/4);
* a product w * h is taken as floor((w H + 2^(s-1)) / 2^s), the 64-bit
  product rounded half up to an integer, then wrapped to 32 bits.

So the output is the exact DFT of the integer input, up to the rounding of
the products (and the rounding of the constants), as long as no value
leaves the 32-bit range; the GPU path computes the same integers bit for bit.

``cdft_fixed`` is the integer transform.  ``cdft_model`` runs the very same
code on FP64 values: with ``noise=None`` every product is exact (w * h), so it
must agree with the FP64 oracle ``oracle/qft.py`` to rounding (this pins the
structure); with a random generator it adds an independent uniform error in
[-1/2, 1/2) after every product (the rounding model of the integer mode).
"""
import math

import numpy as np

__all__ = ["secant_table_q", "cdft_fixed", "cdft_model", "products_per_transform"]

_M32 = (1 << 32) - 1


def _slice(L):
    """Mantissas (int64 array) and shift of the constants of periodization 8L."""
    h = [1.0 / (2.0 * math.cos(math.pi * (2 * m + 1) / (4 * L))) for m in range(L)]
    e = math.frexp(h[-1])[1]
    s = 30 - e
    H = np.array([math.floor(v * 2.0 ** s + 0.5) for v in h], dtype=np.int64)
    return h, H, s


def secant_table_q(log2n_max):
    """Integer constant table for N up to 2^log2n_max, laid out like the FP32
    table of the GPU path: entry L + m (L = 1, 2, .., N/8; m < L) holds
    H_L(m); shifts[L] = s_L.  Entry 0 is unused (0).  Returns (H, shifts)
    as int64 arrays of N/4 entries."""
    nt = max((1 << log2n_max) // 4, 2)
    H = np.zeros(nt, dtype=np.int64)
    shifts = np.zeros(nt, dtype=np.int64)
    L = 1
    while 2 * L <= nt:
        _, h, s = _slice(L)
        H[L:2 * L] = h
        shifts[L] = s
        L *= 2
    return H, shifts


# --------------------------------------------------------------------------
# Arithmetic backends: integers (wrapping) or FP64 (exact or with the
# rounding model)
# --------------------------------------------------------------------------
class _Int:
    def __init__(self):
        self.cache = {}

    @staticmethod
    def wrap(v):
        return ((v + (1 << 31)) & _M32) - (1 << 31)

    def add(self, a, b):
        return self.wrap(a + b)

    def sub(self, a, b):
        return self.wrap(a - b)

    def neg(self, a):
        return self.wrap(-a)

    def mul(self, w, L):
        """w (last axis: m = 0..L-1) times h_L(m), rounded as stated."""
        if L not in self.cache:
            self.cache[L] = _slice(L)[1:]
        H, s = self.cache[L]
        return self.wrap((w * H + (1 << (s - 1))) >> s)


class _Float:
    def __init__(self, rng=None):
        self.rng = rng
        self.cache = {}

    @staticmethod
    def add(a, b):
        return a + b

    @staticmethod
    def sub(a, b):
        return a - b

    @staticmethod
    def neg(a):
        return -a

    def mul(self, w, L):
        if L not in self.cache:
            self.cache[L] = np.array(_slice(L)[0])
        t = w * self.cache[L]
        if self.rng is not None:
            t = t + (self.rng.random(t.shape) - 0.5)
        return t


# --------------------------------------------------------------------------
# The DCT family (Sec. 5.2.1 - 5.2.3), stored samples on the last axis
# --------------------------------------------------------------------------
def _dct(A, s, N):
    """``dct``: s_dc_tt, n = 0..N/2 -> DCT-0, k = 0..N/2."""
    if N == 2:
        return np.stack([A.add(s[..., 0], s[..., 1]), A.sub(s[..., 0], s[..., 1])], axis=-1)
    q = N // 4
    E = _dct(A, s[..., 0::2], N // 2)          # even n, halved (Sec. 3.4)
    O = _dct_ot(A, s[..., 1::2], N)            # odd n
    S = np.empty(s.shape[:-1] + (N // 2 + 1,), dtype=s.dtype)
    S[..., 0:q] = A.add(E[..., 0:q], O)        # eq. qft_5C
    S[..., N // 2:q:-1] = A.sub(E[..., 0:q], O)  # eq. qft_5D
    S[..., q] = E[..., q]                      # eq. qft_6
    return S


def _dct_ot(A, s, N):
    """``dct_ot``: s_dc_ot, n = 1,3,..,N/2-1 -> k = 0..N/4-1."""
    if N == 4:
        return s.copy()
    m = N // 8
    a, b = s[..., :m], s[..., ::-1][..., :m]   # s(n), s(N/2 - n)
    E = _dct_ot(A, A.add(a, b), N // 2)        # even k (Sec. 3.2, 3.3)
    O = _dct_oo(A, A.sub(a, b), N)             # odd k
    S = np.empty(s.shape[:-1] + (N // 4,), dtype=s.dtype)
    S[..., 0::2] = E                           # eq. qft_4B
    S[..., 1::2] = O
    return S


def _dct_oo(A, s, N):
    """``dct_oo``: s_dc_oo, n = 1,3,..,N/4-1 -> odd k = 1,3,..,N/4-1."""
    if N == 8:
        return A.mul(s, 1)                     # x cos(pi/4), slice L = 1
    t = A.mul(s, N // 8)                       # eq. qft_38A
    T = _dct_ot(A, t, N // 2)
    S = np.empty_like(T)
    S[..., :-1] = A.add(T[..., :-1], T[..., 1:])  # eq. qft_38C, corrected 38B
    S[..., -1] = T[..., -1]
    return S


# --------------------------------------------------------------------------
# The DST family (Sec. 5.2.4)
# --------------------------------------------------------------------------
def _dst(A, s, N):
    """``dst``: s_ds_tt, n = 1..N/2-1 (stored at n-1) -> k = 1..N/2-1."""
    if N == 4:
        return s.copy()
    q = N // 4
    E = _dst(A, s[..., 1::2], N // 2)          # n = 2, 4, ..
    O = _dst_ot(A, s[..., 0::2], N)            # n = 1, 3, ..
    S = np.empty(s.shape[:-1] + (N // 2 - 1,), dtype=s.dtype)
    S[..., 0:q - 1] = A.add(O[..., 0:q - 1], E)
    S[..., N // 2 - 2:q - 1:-1] = A.sub(O[..., 0:q - 1], E)
    S[..., q - 1] = O[..., q - 1]
    return S


def _dst_ot(A, s, N):
    """``dst_ot``: s_ds_ot, n = 1,3,..,N/2-1 -> k = 1..N/4 (stored at k-1)."""
    if N == 4:
        return s.copy()
    m = N // 8
    a, b = s[..., :m], s[..., ::-1][..., :m]
    E = _dst_ot(A, A.sub(a, b), N // 2)        # even k: the difference (DST swap)
    O = _dst_oo(A, A.add(a, b), N)             # odd k: the sum
    S = np.empty(s.shape[:-1] + (N // 4,), dtype=s.dtype)
    S[..., 1::2] = E
    S[..., 0::2] = O
    return S


def _dst_oo(A, s, N):
    """``dst_oo``: s_ds_oo, n = 1,3,..,N/4-1 -> odd k = 1,3,..,N/4-1."""
    if N == 8:
        return A.mul(s, 1)                     # x sin(pi/4), slice L = 1
    t = A.mul(s, N // 8)
    T = _dst_ot(A, t, N // 2)
    S = np.empty_like(T)
    S[..., 0] = T[..., 0]                      # k = 1: DST[s_oe](0) = 0
    S[..., 1:] = A.add(T[..., :-1], T[..., 1:])
    return S


# --------------------------------------------------------------------------
# rdft and cdft (Sec. 4.2, 4.1)
# --------------------------------------------------------------------------
def _rdft(A, s, N):
    """(C(k), k = 0..N/2; S(k), k = 1..N/2-1) with Re X = C, Im X = -S."""
    if N == 2:
        return np.stack([A.add(s[..., 0], s[..., 1]), A.sub(s[..., 0], s[..., 1])], -1), None
    h = N // 2
    fwd, rev = s[..., 1:h], s[..., :h:-1]      # s(n), s(N - n)
    c = np.empty(s.shape[:-1] + (h + 1,), dtype=s.dtype)
    c[..., 0] = s[..., 0]
    c[..., h] = s[..., h]
    c[..., 1:h] = A.add(fwd, rev)
    d = A.sub(fwd, rev)
    return _dct(A, c, N), _dst(A, d, N)


def _cdft(A, re, im):
    N = re.shape[-1]
    h = N // 2
    Cr, Sr = _rdft(A, re, N)
    Ci, Si = _rdft(A, im, N)
    Xr = np.empty(re.shape, dtype=re.dtype)
    Xi = np.empty(re.shape, dtype=re.dtype)
    Xr[..., 0], Xi[..., 0] = Cr[..., 0], Ci[..., 0]
    Xr[..., h], Xi[..., h] = Cr[..., h], Ci[..., h]
    if N > 2:
        # X(k) = C(k) - i S(k) per real part: Re X(k) = Cr + Si, Im X(k) = Ci - Sr,
        # X(N-k) = C(k) + i S(k): Re = Cr - Si, Im = Ci + Sr   (k = 1..N/2-1)
        cr, ci = Cr[..., 1:h], Ci[..., 1:h]
        Xr[..., 1:h] = A.add(cr, Si)
        Xi[..., 1:h] = A.sub(ci, Sr)
        Xr[..., N - 1:h:-1] = A.sub(cr, Si)
        Xi[..., N - 1:h:-1] = A.add(ci, Sr)
    return Xr, Xi


def cdft_fixed(x):
    """Integer improved QFT of complex integer signals.

    x: integer array [..., N, 2] (real, imaginary), values taken modulo 2^32
    as signed 32-bit integers; N = 2^r, r >= 1.  Returns int64 [..., N, 2]
    holding the signed 32-bit results."""
    x = np.asarray(x, dtype=np.int64)
    N = x.shape[-2]
    if N < 2 or (N & (N - 1)) or x.shape[-1] != 2:
        raise ValueError("x must be [..., N, 2] with N a power of two >= 2")
    A = _Int()
    re, im = _Int.wrap(x[..., 0]), _Int.wrap(x[..., 1])
    Xr, Xi = _cdft(A, np.ascontiguousarray(re), np.ascontiguousarray(im))
    return np.stack([Xr, Xi], axis=-1)


def cdft_model(x, rng=None):
    """The same recursion on FP64 values (complex [..., N] in and out): exact
    products if rng is None, else each product plus uniform noise in [-1/2,
    1/2) drawn from rng (the rounding model of cdft_fixed)."""
    x = np.asarray(x, dtype=np.complex128)
    A = _Float(rng)
    Xr, Xi = _cdft(A, np.ascontiguousarray(x.real), np.ascontiguousarray(x.imag))
    return Xr + 1j * Xi


def products_per_transform(N):
    """Number of rounded products in one complex transform of length N (the
    multiplication count of Table 2, CDFT row: N log2 N - 3N + 4)."""
    r = int(N).bit_length() - 1
    return N * r - 3 * N + 4 if N >= 4 else 0
