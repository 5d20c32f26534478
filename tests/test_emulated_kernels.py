"""The GPU kernels' source, run on the CPU, against the FP64 oracle.

tests/emu/qft_emu.cpp compiles the unchanged kernel bodies
(paper_1301_0763_amd/csrc/qft_device.hpp) and host schedules
(qft_schedule.hpp) for the host and runs each workgroup as OS threads with a
barrier.  Every LDS and heap-buffer access is tracked: a cell written by one
thread and touched by another between two barriers is a race.  These tests
need no GPU; they check indexing, barriers and the multi-pass/uneven
schedules (with small segment sizes, so that many passes occur at small N).

Tolerance: FP32 arithmetic, relative RMS error (eq. qft_44 per signal)
<= 1e-5 * log2 N against the FP64 oracle run on the FP32-rounded input.
"""
import ctypes

import numpy as np
import pytest

import workloads
from oracle import build as OB
from oracle import direct as D
from oracle import qft as Q
from tests.emu import build as EB


@pytest.fixture(scope="module")
def emu():
    return EB.load()


def _as_c64(x):
    return np.ascontiguousarray(x.astype(np.complex64))


@pytest.mark.parametrize("order,same_wave,expect_race", [
    (0, 1, True),   # no ordering at all
    (0, 0, True),
    (1, 1, False),  # a wave-level sync orders the lanes of one wavefront
    (1, 0, True),   # ... but not two wavefronts
    (2, 1, False),  # a workgroup barrier orders everything
    (2, 0, False),
])
def test_race_model(emu, order, same_wave, expect_race):
    """The emulator's race tracker: a write and a read of one cell by two
    threads race unless a workgroup barrier lies between them, or a
    wave-level sync and both threads are lanes of one wavefront."""
    races = emu.emu_race_model_check(order, same_wave)
    assert (races > 0) == expect_race, races


def _tol(logn):
    return 1e-5 * logn


def _ref(x64, swap=False):
    x = x64.astype(np.complex128)
    if x.shape[-1] >= 4096:
        X = OB.cdft(np.conj(x) if swap else x)
        return np.conj(X) if swap else X
    return Q.qft_adjoint(x) if swap else Q.qft(x)


def run_mp(emu, x, seg, nthr=16, swap=0):
    xf = _as_c64(x)
    out = np.zeros_like(xf)
    B, N = xf.shape
    races = emu.emu_multipass(0, swap, xf.ctypes.data, out.ctypes.data, N.bit_length() - 1, B,
                              seg, nthr)
    assert races >= 0, races
    return races, out


@pytest.mark.parametrize("seg,logn", [(3, 6), (3, 9), (4, 7), (4, 11), (5, 8), (5, 12),
                                      (3, 12), (4, 13), (3, 14)])
def test_multipass_small_segments(emu, seg, logn):
    """The multi-pass schedule with segments of 2^seg cells (the library uses
    2^12), so that the global forward/backward rounds and chain levels occur
    at small N; the cases cover passes of 1 to 5 rounds or chain levels, one
    to three chain passes, and the race tracker checks that the in-place
    chain passes and the grouped backward passes touch no cell another item
    of the same pass writes."""
    x = workloads.normal(seg * 100 + logn, (2, 1 << logn))
    races, out = run_mp(emu, x, seg)
    assert races == 0
    assert D.relative_l2(out, _ref(x)).max() <= _tol(logn)


def test_multipass_adjoint(emu):
    x = workloads.uniform(5, (2, 1 << 10))
    races, out = run_mp(emu, x, 4, swap=1)
    assert races == 0
    assert D.relative_l2(out, _ref(x, swap=True)).max() <= _tol(10)


@pytest.mark.slow
def test_multipass_library_segment_size(emu):
    """N = 2^15 with the library's 2^12-cell segments, and N = 2^16 with its
    2^13-cell ones (the "/s13" schedules) bit-identical to 2^12-cell ones."""
    x = workloads.normal(15, (1, 1 << 15))
    races, out = run_mp(emu, x, 12, nthr=64)
    assert races == 0
    assert D.relative_l2(out, _ref(x)).max() <= _tol(15)
    x = workloads.normal(16, (1, 1 << 16))
    races, out12 = run_mp(emu, x, 12, nthr=64)
    assert races == 0
    races, out13 = run_mp(emu, x, 13, nthr=64)
    assert races == 0
    assert np.array_equal(out12, out13)
    assert D.relative_l2(out13, _ref(x)).max() <= _tol(16)


def test_uneven_worklist(emu):
    """Packed uneven batch as the library runs it: sizes up to 2^10 share
    2^10-cell tiles of the size-sorted work list, 2^11 .. 2^14 take a tile of
    their own, all through the specialised tile kernel and the offset list;
    2^15 goes through the two-pass path (2^12-cell segments, the library's
    threads), 2^17 multi-pass (segments of 2^3 here)."""
    rng = np.random.default_rng(3)
    log2n = np.array(list(rng.integers(1, 13, 40)) + [13, 14, 15, 17], dtype=np.int32)
    rng.shuffle(log2n)
    total = int(np.sum(1 << log2n.astype(np.int64)))
    vals = workloads.uniform(21, (total,))
    xf = _as_c64(vals)
    out = np.zeros_like(xf)
    races = emu.emu_uneven(0, 0, xf.ctypes.data, out.ctypes.data,
                           log2n.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), log2n.size,
                           3, 16)
    assert races == 0
    off = 0
    for r in log2n:
        N = 1 << int(r)
        seg = xf[off:off + N][None]
        err = D.relative_l2(out[off:off + N][None], _ref(seg)).max()
        assert err <= _tol(max(int(r), 1)), (r, err)
        off += N


def run_tp(emu, x, mc_log2, swap=0, grid=0):
    xf = _as_c64(x)
    out = np.zeros_like(xf)
    races = emu.emu_twopass(0, swap, xf.ctypes.data, out.ctypes.data, mc_log2, xf.shape[0],
                            grid)
    assert races >= 0, races
    return races, out


@pytest.mark.parametrize("mc_log2", [3, 4, 5, 7, 10])
@pytest.mark.parametrize("swap", [0, 1])
def test_two_pass_small(emu, mc_log2, swap):
    """Two-pass path (N = 8 * segment) with small segments: pass A gathers
    both sides of a segment with the fold and the top round from x, runs the
    segment's remaining rounds (and, for the head, the DCT-0/DST-0 chain up to
    P = 2 * segment) in LDS; pass B streams the top backward round, chain
    levels N/2 and N and the combine.  The race tracker checks that no two
    workgroups of pass A write one heap cell."""
    logn = mc_log2 + 3
    x = workloads.normal(500 + mc_log2, (3, 1 << logn))
    races, out = run_tp(emu, x, mc_log2, swap=swap)
    assert races == 0
    assert D.relative_l2(out, _ref(x, swap=bool(swap))).max() <= _tol(logn)


@pytest.mark.parametrize("logn,seg", [(12, 3), (14, 5)])
def test_multipass_level_splits_agree(emu, logn, seg):
    """Every split of the global passes that a multi-pass plan offers as a
    schedule (most forward rounds / backward rounds / chain levels per pass)
    computes the same rounds and levels: bit-identical results."""
    x = _as_c64(workloads.normal(700 + logn, (2, 1 << logn)))
    outs = []
    for f, b, c in [(4, 5, 5), (3, 5, 5), (4, 4, 5), (4, 5, 4), (3, 4, 4), (5, 5, 5), (1, 1, 1)]:
        out = np.zeros_like(x)
        races = emu.emu_multipass_levels(0, x.ctypes.data, out.ctypes.data, logn, 2, seg, 32,
                                         f, b, c)
        assert races == 0, (f, b, c, races)
        outs.append(out)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    assert D.relative_l2(outs[0], _ref(x)).max() <= _tol(logn)


@pytest.mark.parametrize("mc_log2,batch", [(3, 19), (5, 11), (7, 9), (10, 17)])
@pytest.mark.parametrize("grid", [32, 64])
def test_two_pass_persistent(emu, mc_log2, batch, grid):
    """Persistent pass A (a grid of whole groups of 32 workgroups, each taking
    every grid-th tile): bit-identical to one workgroup per tile, on batches
    whose last group of eight transforms is ragged, and race free."""
    logn = mc_log2 + 3
    x = workloads.normal(600 + mc_log2, (batch, 1 << logn))
    r0, ref = run_tp(emu, x, mc_log2)
    r1, out = run_tp(emu, x, mc_log2, grid=grid)
    assert r0 == 0 and r1 == 0
    assert np.array_equal(out, ref)
    assert D.relative_l2(out, _ref(x)).max() <= _tol(logn)


@pytest.mark.slow
def test_two_pass_library_size(emu):
    """N = 2^15 and 2^16 with the library's 2^12- and 2^13-cell segments and
    thread counts, one workgroup per tile and persistent."""
    for mc in (12, 13):
        x = workloads.normal(15, (9, 8 << mc))
        races, out = run_tp(emu, x, mc)
        assert races == 0
        assert D.relative_l2(out, _ref(x)).max() <= _tol(mc + 3)
        races, pout = run_tp(emu, x, mc, grid=32)
        assert races == 0 and np.array_equal(pout, out)


@pytest.mark.parametrize("logn,batch,grid", [(1, 1100, 2), (4, 200, 3), (7, 19, 2), (10, 5, 2),
                                             (11, 7, 3), (12, 5, 2), (13, 3, 2), (14, 3, 2)])
@pytest.mark.parametrize("swap", [0, 1])
def test_resident_grid_tiles(emu, logn, batch, grid, swap):
    """The resident-grid tile kernel (each workgroup strides over the tiles
    and loads its next tile's x while the current one runs its rounds):
    bit-identical to one workgroup per tile, with several tiles per
    workgroup, a ragged last tile and workgroups without one; race free."""
    N = 1 << logn
    T = max(1, 1024 // N)
    x = _as_c64(workloads.uniform(900 + logn, (batch, N)))
    ref = np.zeros_like(x)
    for t0 in range(0, batch, T):
        cnt = min(T, batch - t0)
        sub = np.ascontiguousarray(x[t0:t0 + cnt])
        o = np.zeros_like(sub)
        assert emu.emu_tile_s(0, swap, sub.ctypes.data, o.ctypes.data, logn, cnt, None) == 0
        ref[t0:t0 + cnt] = o
    out = np.zeros_like(x)
    assert emu.emu_tile_p(0, swap, x.ctypes.data, out.ctypes.data, logn, batch, grid) == 0
    assert np.array_equal(out, ref)
    # more workgroups than tiles: the extra ones exit at once
    ntiles = -(-batch // T)
    out2 = np.zeros_like(x)
    assert emu.emu_tile_p(0, swap, x.ctypes.data, out2.ctypes.data, logn, batch,
                          ntiles + 1) == 0
    assert np.array_equal(out2, ref)


@pytest.mark.parametrize("logn", [13, 14])
@pytest.mark.parametrize("swap", [0, 1])
def test_resident_grid_uneven_list(emu, logn, swap):
    """The resident-grid kernel of an uneven group of one-transform tiles:
    it walks the group's tile list (tiles in a different order than the
    transforms lie in memory, between transforms of other sizes), resolves
    each transform's offset once per tile and loads the next tile during the
    current one; bit-identical to the tile kernel on each transform."""
    N = 1 << logn
    rng = np.random.default_rng(31 + logn)
    count = 5
    gaps = rng.integers(1, 300, count)  # other transforms' points between them
    offs = np.cumsum(gaps + np.r_[0, np.full(count - 1, N)]).astype(np.int64)
    total = int(offs[-1] + N + 17)
    x = _as_c64(workloads.uniform(950 + logn, (1, total)))[0]
    order = rng.permutation(count)
    tiles = np.zeros((count, 4), np.int32)
    tiles[:, 0] = logn
    tiles[:, 1] = order
    tiles[:, 2] = 1
    out = np.zeros_like(x)
    assert emu.emu_tile_pg(0, swap, x.ctypes.data, out.ctypes.data, logn, tiles.ctypes.data,
                           offs.ctypes.data, count, 2) == 0
    untouched = np.ones(total, bool)
    for o in offs:
        seg = np.ascontiguousarray(x[o:o + N][None])
        ref = np.zeros_like(seg)
        assert emu.emu_tile_s(0, swap, seg.ctypes.data, ref.ctypes.data, logn, 1, None) == 0
        assert np.array_equal(out[o:o + N], ref[0])
        untouched[o:o + N] = False
    assert not out[untouched].any()


@pytest.mark.parametrize("logn", range(1, 15))
def test_specialised_tile_as_launched(emu, logn):
    """The compile-time specialised tile kernel with the GPU's own tile size
    and thread count (2^10-cell tiles of 64 threads up to N = 2^10, then one
    transform per tile with 128 or 256 threads of 16 cells, or 256 or 512 of
    32 cells for 2^13 and 2^14), on a full tile and on a ragged last tile."""
    N = 1 << logn
    T = max(1, 1024 // N)  # transforms per tile: 2^max(10, logn) cells
    for Tact in sorted({T, max(1, T // 2 - 1)}):
        x = workloads.uniform(700 + logn + Tact, (Tact, N))
        xf = _as_c64(x)
        out = np.zeros_like(xf)
        races = emu.emu_tile_s(0, 0, xf.ctypes.data, out.ctypes.data, logn, Tact, None)
        assert races == 0, races
        assert D.relative_l2(out, _ref(x)).max() <= _tol(max(logn, 1))


@pytest.mark.parametrize("logn", [2, 9, 13])
def test_specialised_tile_adjoint_and_fp16(emu, logn):
    N = 1 << logn
    x = workloads.uniform(800 + logn, (1, N))
    xf = _as_c64(x)
    out = np.zeros_like(xf)
    assert emu.emu_tile_s(0, 1, xf.ctypes.data, out.ctypes.data, logn, 1, None) == 0
    assert D.relative_l2(out, _ref(x, swap=True)).max() <= _tol(logn)
    x16 = np.stack([x.real, x.imag], -1).astype(np.float16)
    o16 = np.zeros_like(x16)
    assert emu.emu_tile_s(1, 0, x16.ctypes.data, o16.ctypes.data, logn, 1, None) == 0
    xin = x16[..., 0].astype(np.float64) + 1j * x16[..., 1].astype(np.float64)
    got = o16[..., 0].astype(np.float64) + 1j * o16[..., 1].astype(np.float64)
    assert D.relative_l2(got, Q.qft(xin)).max() < 1e-3


@pytest.mark.parametrize("logn", [3, 7, 10, 12])
@pytest.mark.parametrize("swap", [0, 1])
def test_specialised_tile_offset_list(emu, logn, swap):
    """The persistent kernel of uneven plans: the same specialised body with
    transform t read from and written to element offset offs[t] (here a
    scrambled order with gaps that other transforms' data fill)."""
    N = 1 << logn
    T = max(1, 1024 // N)  # transforms per tile: 2^max(10, logn) cells
    Tact = max(1, T - 1)
    rng = np.random.default_rng(logn)
    slots = rng.permutation(Tact + 2)[:Tact]  # transforms at scattered slots
    offs = np.ascontiguousarray((slots * N).astype(np.int64))
    x = workloads.uniform(900 + logn, ((Tact + 2) * N,))
    xf = _as_c64(x)
    out = np.full_like(xf, np.nan)
    races = emu.emu_tile_s(0, swap, xf.ctypes.data, out.ctypes.data, logn, Tact,
                           offs.ctypes.data)
    assert races == 0
    sig = np.stack([x[o:o + N] for o in offs])
    got = np.stack([out[o:o + N] for o in offs])
    assert D.relative_l2(got, _ref(sig, swap=bool(swap))).max() <= _tol(logn)
    # slots that hold no transform of the tile are left untouched
    free = np.setdiff1d(np.arange(Tact + 2), slots)
    assert np.all(np.isnan(out[free[0] * N:(free[0] + 1) * N]))


def _ptr(a):
    return None if a is None else a.ctypes.data


@pytest.mark.parametrize("logn", [1, 2, 3, 5, 8, 10, 12, 13])
@pytest.mark.parametrize("odd", [0, 1])
def test_specialised_tile_real_input(emu, logn, odd):
    """Real-input tile: two real signals per transform slot (lanes x, y), the
    half spectrum X(k) = C(k) - i S(k), k = 0..N/2 of each (rdft, Sec. 4.2),
    against the oracle's rdft; an odd number of signals leaves the last
    slot's second lane empty."""
    N = 1 << logn
    T = max(1, 1024 // N)  # transforms per tile: 2^max(10, logn) cells
    rows = min(2 * T, 6) - odd
    x = np.ascontiguousarray(workloads.normal(1200 + logn, (rows, N)).real.astype(np.float32))
    out = np.full((rows, N // 2 + 1), np.nan + 1j * np.nan, dtype=np.complex64)
    races = emu.emu_tile_real(0, 0, logn, rows, _ptr(x), None, _ptr(out), None)
    assert races == 0, races
    re, im = Q.rdft(x.astype(np.float64), N, Q.Ops())
    ref = re.astype(np.complex128)
    if N > 2:
        ref[..., 1:N // 2] += 1j * im
    assert D.relative_l2(out.astype(np.complex128), ref).max() <= _tol(logn)
    # and the definition of the half spectrum
    np.testing.assert_allclose(out, np.fft.fft(x.astype(np.float64))[..., :N // 2 + 1],
                               rtol=0, atol=_tol(logn) * np.sqrt(N) * 4)


@pytest.mark.parametrize("logn", [1, 2, 3, 4, 6, 9, 12])
@pytest.mark.parametrize("which", ["both", "dct", "dst"])
def test_specialised_tile_dct0_dst0(emu, logn, which):
    """DCT-0 and DST-0 entry point: the heap fed straight with c(n) and d(n),
    C(k) and S(k) read out unfolded, against the oracle's dct and dst."""
    N = 1 << logn
    h = N // 2
    if which == "dst" and h - 1 == 0:
        pytest.skip("the DST-0 of N = 2 is empty")
    T = max(1, 1024 // N)  # transforms per tile: 2^max(10, logn) cells
    rows = min(5, 2 * T)
    c = np.ascontiguousarray(workloads.uniform(1300 + logn, (rows, h + 1)).real.astype(np.float32))
    d = np.ascontiguousarray(workloads.uniform(1400 + logn, (rows, max(h - 1, 1))).real
                             .astype(np.float32)[:, :h - 1])
    C = np.full((rows, h + 1), np.nan, np.float32)
    S = np.full((rows, max(h - 1, 0)), np.nan, np.float32)
    use_c, use_d = which in ("both", "dct"), which in ("both", "dst") and h > 1
    races = emu.emu_tile_real(1, 0, logn, rows, _ptr(c) if use_c else None,
                              _ptr(d) if use_d else None, _ptr(C) if use_c else None,
                              _ptr(S) if use_d else None)
    assert races == 0, races
    if use_c:
        refC = Q.dct(c.astype(np.float64), N, Q.Ops())
        assert D.relative_l2(C.astype(np.float64), refC).max() <= _tol(logn)
    else:
        assert np.all(np.isnan(C))
    if use_d:
        refS = Q.dst(d.astype(np.float64), N, Q.Ops())
        assert D.relative_l2(S.astype(np.float64), refS).max() <= _tol(logn)
    elif h > 1:
        assert np.all(np.isnan(S))


@pytest.mark.parametrize("seg,logn", [(3, 6), (4, 9), (5, 11)])
@pytest.mark.parametrize("rows", [3, 4])
def test_multipass_real_input(emu, seg, logn, rows):
    """Real-input plans longer than a tile: the multi-pass schedule (small
    segments so that every global stage occurs) with the real fold and the
    half-spectrum / DCT-0 / DST-0 read-out."""
    N, h = 1 << logn, 1 << (logn - 1)
    x = np.ascontiguousarray(workloads.normal(1500 + logn, (rows, N)).real.astype(np.float32))
    out = np.zeros((rows, h + 1), np.complex64)
    assert emu.emu_multipass_real(0, 0, logn, rows, _ptr(x), None, _ptr(out), None, seg, 16) == 0
    assert D.relative_l2(out.astype(np.complex128), _rdft_emu_ref(x)).max() <= _tol(logn)
    c = np.ascontiguousarray(workloads.uniform(1600 + logn, (rows, h + 1)).real.astype(np.float32))
    d = np.ascontiguousarray(workloads.uniform(1700 + logn, (rows, h - 1)).real.astype(np.float32))
    C = np.zeros_like(c)
    S = np.zeros_like(d)
    assert emu.emu_multipass_real(1, 0, logn, rows, _ptr(c), _ptr(d), _ptr(C), _ptr(S), seg,
                                  16) == 0
    assert D.relative_l2(C.astype(np.float64), Q.dct(c.astype(np.float64), N, Q.Ops())).max() \
        <= _tol(logn)
    assert D.relative_l2(S.astype(np.float64), Q.dst(d.astype(np.float64), N, Q.Ops())).max() \
        <= _tol(logn)


def _rdft_emu_ref(x):
    N = x.shape[-1]
    re, im = Q.rdft(x.astype(np.float64), N, Q.Ops())
    ref = re.astype(np.complex128)
    ref[..., 1:N // 2] += 1j * im
    return ref


@pytest.mark.parametrize("logn", list(range(1, 12)) + [13])
def test_fixed_point_emulated(emu, logn):
    """The fixed-point kernel body (qft_fixed.hpp) run on the CPU with the
    library's threads per transform (and with 64 or 256), forward rounds one or
    two per pass: bit-identical to the integer oracle, including inputs that
    overflow (two's complement wrap), and race free.  With at most 64 threads
    the passes are ordered by wavefront syncs only, as the GPU runs transforms
    of up to 2^8 points."""
    from oracle import qft_fixed as F
    N = 1 << logn
    # the GPU's threads per transform: N/4 within [64, 1024], and for N < 2^12
    # at most 1024 / (2^12 / N) (several transforms per workgroup)
    g = min(max(N // 4, 64), 1024)
    if logn < 12:
        t = min(1 << (12 - logn), 1024)
        g = min(g, 1024 // t)
    rng = np.random.default_rng(900 + logn)
    for nthr in sorted({g, 64 if logn <= 9 else 256}):
        for fuse2 in (0, 1):
            for lim in (1 << (28 - logn), 1 << 31):
                x = rng.integers(-lim, lim, (2, N, 2)).astype(np.int32)
                X = np.zeros_like(x)
                races = emu.emu_fixed(x.ctypes.data, X.ctypes.data, logn, 2, nthr, fuse2)
                assert races == 0, (nthr, fuse2)
                assert np.array_equal(X.astype(np.int64), F.cdft_fixed(x)), (nthr, fuse2)


def test_fixed_point_table_matches_oracle(emu):
    """The library's integer constant table (host code) and the oracle's,
    computed independently from the same definition, are identical."""
    from oracle import qft_fixed as F
    for r in (3, 8, 12, 16):
        nt = (1 << r) // 4
        H = np.zeros(nt, np.int32)
        sh = np.zeros(32, np.int32)
        assert emu.emu_fixed_table(r, H.ctypes.data, sh.ctypes.data) == 0
        Ho, so = F.secant_table_q(r)
        assert np.array_equal(H.astype(np.int64), Ho)
        L, lg = 1, 0
        while 2 * L <= nt:
            assert sh[lg] == so[L]
            L, lg = 2 * L, lg + 1
