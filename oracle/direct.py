"""Oracle A: the complex DFT by its definition, in FP64.

Test infrastructure only (see ``oracle/__init__``).

Definition followed (Pasquini, Sec. 2.1, eq. qft_0A with eq. qft_0D):

    X(k) = sum_{n=0}^{N-1} x(n) * exp(-i * theta * n * k),  theta = 2*pi/N,
    k = 0..N-1, unnormalised.

The only implementation choice is how exp(-i*theta*m) is evaluated. The angle
index is reduced exactly in integers, m = (n*k) mod N, and the unit roots are
built from angles in [0, pi/4] by the octant symmetries of sine and cosine, so
no large-argument trigonometry is ever evaluated.

``dft_adjoint`` is the conjugate transpose (exp(+i...)), i.e. the map that the
backward/adjoint entry point computes.
"""
import numpy as np

__all__ = ["unit_roots", "dft", "dft_bins", "dft_adjoint", "relative_l2", "bin_errors"]


def unit_roots(N):
    """w[m] = exp(-2*pi*i*m/N), m = 0..N-1, FP64.

    The angle a = 2*pi*m/N = (pi/4)*(8m/N) is split exactly in integers into an
    octant index o = floor(8m/N) and a residual, so that sine and cosine are only
    ever evaluated on [0, pi/4]; the octant is restored by quarter-turn rotations.
    Indices above N/2 are taken as conjugates of their mirror N - m.
    """
    N = int(N)
    m = np.arange(N, dtype=np.int64)
    eighth = 8 * m
    octant = eighth // N
    rem = eighth - octant * N
    unit = 2.0 * np.pi / (8.0 * N)
    odd = (octant % 2) == 1
    b = np.where(odd, unit * (N - rem), unit * rem)
    c = np.cos(b)
    s = np.where(odd, -np.sin(b), np.sin(b))
    base = np.where(odd, (octant + 1) // 2, octant // 2) % 4
    # rotation by base*pi/2: (c, s) -> (-s, c) per step
    c1, s1 = c.copy(), s.copy()
    for k in (1, 2, 3):
        sel = base == k
        cc, ss = c[sel], s[sel]
        if k == 1:
            c1[sel], s1[sel] = -ss, cc
        elif k == 2:
            c1[sel], s1[sel] = -cc, -ss
        else:
            c1[sel], s1[sel] = ss, -cc
    w = c1 - 1j * s1
    # exact conjugate symmetry: exp(-2 pi i (N-m)/N) = conj(exp(-2 pi i m/N))
    upper = m[2 * m > N]
    w[upper] = np.conj(w[N - upper])
    return w


def dft_bins(x, bins, sign=-1):
    """X(k) for the listed bins k only (each bin is O(N)). x: [..., N]."""
    x = np.asarray(x, dtype=np.complex128)
    N = x.shape[-1]
    w = unit_roots(N)
    if sign > 0:
        w = np.conj(w)
    bins = np.asarray(bins, dtype=np.int64)
    n = np.arange(N, dtype=np.int64)
    out = np.empty(x.shape[:-1] + (bins.size,), dtype=np.complex128)
    step = max(1, (1 << 22) // max(N, 1))
    for i0 in range(0, bins.size, step):
        kb = bins[i0:i0 + step]
        idx = (np.outer(kb, n) % N)
        out[..., i0:i0 + kb.size] = x @ w[idx].T
    return out


def dft(x):
    """Full unnormalised forward DFT of the last axis (O(N^2) per signal)."""
    x = np.asarray(x, dtype=np.complex128)
    return dft_bins(x, np.arange(x.shape[-1]), sign=-1)


def dft_adjoint(X):
    """Conjugate-transpose map: x(n) = sum_k X(k) exp(+2*pi*i*n*k/N)."""
    X = np.asarray(X, dtype=np.complex128)
    return dft_bins(X, np.arange(X.shape[-1]), sign=+1)


def relative_l2(S, S_exact, axis=-1):
    """Per-signal ||S - S_exact||_2 / ||S_exact||_2 (the accuracy measure of
    Sec. 6.3, eq. qft_44, before averaging over signals)."""
    S = np.asarray(S, dtype=np.complex128)
    S_exact = np.asarray(S_exact, dtype=np.complex128)
    num = np.sqrt(np.sum(np.abs(S - S_exact) ** 2, axis=axis))
    den = np.sqrt(np.sum(np.abs(S_exact) ** 2, axis=axis))
    return num / den


def bin_errors(S, S_exact, axis=-1):
    """Per-bin error scaled by the signal's RMS: |S(k) - S_exact(k)| / rms(S_exact),
    rms(S_exact) = sqrt(mean_k |S_exact(k)|^2) over the given axis.  Its maximum
    over k bounds the worst single bin, which the per-signal relative L2 of
    eq. qft_44 averages away (relative_l2 = sqrt(mean_k bin_errors^2))."""
    S = np.asarray(S, dtype=np.complex128)
    S_exact = np.asarray(S_exact, dtype=np.complex128)
    rms = np.sqrt(np.mean(np.abs(S_exact) ** 2, axis=axis, keepdims=True))
    return np.abs(S - S_exact) / rms
