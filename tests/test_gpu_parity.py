"""GPU parity: the gfx950 library (through the C ABI) against the FP64 oracle.

Every comparison goes through ``tests.parity.check`` (bounds derived there):
per signal, the relative L2 error (eq. qft_44 before averaging) is at most
1e-5 * log2 N, and every single bin is within c(n) * 1e-5 * log2 N * rms of
the oracle's value, with X_ref the FP64 oracle evaluated on the stored input.
FP16 storage adds the output rounding (2^-11 relative per element) to the bin
bound and is held to 1e-3 in relative L2.
"""
import ctypes
import json
import sys

import numpy as np
import pytest

import workloads
from oracle import build as OB
from oracle import direct as D
from oracle import qft as Q
from tests.parity import check, tol

torch = pytest.importorskip("torch")
import paper_1301_0763_amd as qft  # noqa: E402
from paper_1301_0763_amd import _lib  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def ref_fwd(x):
    x = np.asarray(x, dtype=np.complex128)
    if x.shape[-1] <= 256:
        return Q.qft(x)
    return OB.cdft(x)


def gpu_fwd(x, adjoint=False):
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    y = qft.fft_adjoint(xt) if adjoint else qft.fft(xt)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def test_c1_against_direct_dft():
    say("c1: N=1024 B=64 U[-1,1] seed 0, fwd vs O(N^2) DFT")
    x = workloads.make("c1")
    X = gpu_fwd(x)
    rel, worst = check(X, D.dft(x.astype(np.complex128)), 10, what="c1")
    say(f"c1 rel-L2 max {rel:.3e}, worst bin {worst:.2f} of its bound")


@pytest.mark.parametrize("logn", range(1, 15))
def test_all_tile_sizes(logn):
    B = 3 if logn > 10 else 5
    say(f"tile sizes: N=2^{logn} B={B}")
    x = workloads.uniform(1000 + logn, (B, 1 << logn))
    check(gpu_fwd(x), ref_fwd(x), logn, what=f"tile 2^{logn}")


@pytest.mark.parametrize("logn,B", [(15, 3), (16, 2), (15, 200), (16, 130), (17, 2), (18, 1),
                                    (19, 1), (20, 2), (21, 1), (22, 1), (23, 1)])
def test_multipass_sizes(logn, B):
    """Two-pass (2^15, 2^16, including batches that leave the last group of
    eight transforms of pass A ragged) and multi-pass sizes: every split of
    the global rounds and chain levels into passes of 3 to 5 that the library
    uses."""
    say(f"multi-pass: N=2^{logn} B={B}")
    x = workloads.normal(2000 + logn, (B, 1 << logn))
    check(gpu_fwd(x), ref_fwd(x), logn, what=f"multi-pass 2^{logn} x {B}")


@pytest.mark.parametrize("logn,B", [(3, 4), (10, 6), (14, 2), (16, 2), (20, 1)])
def test_adjoint_and_round_trip(logn, B):
    say(f"adjoint: N=2^{logn} B={B}")
    x = workloads.uniform(3000 + logn, (B, 1 << logn))
    N = 1 << logn
    y = gpu_fwd(x, adjoint=True)
    ref = np.conj(ref_fwd(np.conj(x.astype(np.complex128))))
    check(y, ref, logn, what="adjoint")
    # bwd(fwd(x)) = N x: two transforms, twice the error budget; relative L2
    # only (the pull-back of the forward's error to x concentrates on a few
    # samples, see tests/parity.py)
    xt = torch.from_numpy(x).to(DEV)
    rt = qft.fft_adjoint(qft.fft(xt)).cpu().numpy() / N
    check(rt, x.astype(np.complex128), 2 * logn, what="round trip", per_bin=False)
    # dot-product test <F x, y> = <x, F^H y>
    z = workloads.uniform(3100 + logn, (B, N))
    Fx = gpu_fwd(x)
    FHz = gpu_fwd(z, adjoint=True)
    lhs = np.vdot(z.astype(np.complex128), Fx)
    rhs = np.vdot(FHz, x.astype(np.complex128))
    assert abs(lhs - rhs) <= tol(logn) * abs(lhs) * 10


@pytest.mark.parametrize("logn,B", [(12, 3), (15, 2), (16, 2), (17, 1), (19, 1)])
def test_fp16_storage_all_paths(logn, B):
    """FP16 storage with FP32 arithmetic on every path (tile, two-pass,
    multi-pass), forward and adjoint, against the FP64 oracle on the
    FP16-rounded input; the output rounding to FP16 bounds the error."""
    say(f"fp16 storage: N=2^{logn} B={B}")
    x = workloads.uniform(9000 + logn, (B, 1 << logn)).astype(np.complex64)
    host = np.stack([x.real, x.imag], -1).astype(np.float16)
    xin = host[..., 0].astype(np.float64) + 1j * host[..., 1].astype(np.float64)
    t = torch.from_numpy(host).to(DEV).view(torch.complex32).reshape(B, -1)
    for adj in (False, True):
        y = qft.fft_adjoint(t) if adj else qft.fft(t)
        torch.cuda.synchronize()
        o = y.view(torch.float16).reshape(B, -1, 2).float().cpu().numpy().astype(np.float64)
        got = o[..., 0] + 1j * o[..., 1]
        ref = np.conj(ref_fwd(np.conj(xin))) if adj else ref_fwd(xin)
        check(got, ref, logn, fp16=True, what=f"fp16 adjoint={adj}")


def test_c2_full_size():
    say("c2: N=2^16 B=256 N(0,1) seed 1 (the benchmark workload), full compare")
    x = workloads.make("c2")
    X = gpu_fwd(x)
    ref = OB.cdft(x.astype(np.complex128))
    rel, worst = check(X, ref, 16, what="c2")
    say(f"c2 rel-L2 max {rel:.3e}, worst bin {worst:.2f} of its bound")
    # independent spot check against the DFT definition on sampled bins
    bins = np.array([0, 1, 7, 4096, 32767, 32768, 32769, 65535])
    direct_vals = D.dft_bins(x[:2].astype(np.complex128), bins)
    scale = np.sqrt(np.mean(np.abs(ref[:2]) ** 2, axis=-1, keepdims=True))
    assert np.max(np.abs(X[:2, bins] - direct_vals) / scale) < 1e-5 * 16


def test_c3_single_large():
    say("c3: N=2^24 B=1 tones+noise seed 2")
    x, freqs, amps = workloads.make("c3")
    X = gpu_fwd(x)
    ref = OB.cdft(x.astype(np.complex128))
    rel, worst = check(X, ref, 24, what="c3")
    say(f"c3 rel-L2 {rel:.3e} (target {tol(24):.1e}), worst bin {worst:.2f} of its bound")
    N = 1 << 24
    # closed form: |X(f_i)| ~ N a_i, far above the noise floor
    got = np.abs(X[0, freqs])
    np.testing.assert_allclose(got, N * amps, rtol=1e-3)


def _uneven(dtype):
    r, vals = workloads.make("c4")
    if dtype == "c16":
        v16 = vals.astype(np.complex64)
        host = np.stack([v16.real, v16.imag], -1).astype(np.float16)
        xin = host[..., 0].astype(np.float64) + 1j * host[..., 1].astype(np.float64)
        t = torch.from_numpy(host).to(DEV).view(torch.complex32).reshape(-1)
    else:
        xin = vals.astype(np.complex128)
        t = torch.from_numpy(vals).to(DEV)
    out = qft.fft_packed(t, r.tolist())
    torch.cuda.synchronize()
    if dtype == "c16":
        o = out.view(torch.float16).reshape(-1, 2).float().cpu().numpy().astype(np.float64)
        got = o[:, 0] + 1j * o[:, 1]
    else:
        got = out.cpu().numpy().astype(np.complex128)
    off = np.concatenate([[0], np.cumsum(1 << r.astype(np.int64))])
    worst = 0.0
    for lg in range(6, 15):
        idx = np.nonzero(r == lg)[0]
        N = 1 << lg
        xs = np.stack([xin[off[i]:off[i] + N] for i in idx])
        gs = np.stack([got[off[i]:off[i] + N] for i in idx])
        rel, _ = check(gs, OB.cdft(xs), lg, fp16=dtype == "c16", what=f"c4 {dtype} 2^{lg}")
        worst = max(worst, rel / (tol(lg) if dtype == "c32" else 1e-3))
    return worst


def test_c4_uneven_fp32():
    say("c4: 4096 uneven transforms r in 6..14, seed 3, FP32")
    assert _uneven("c32") <= 1.0


def test_c4_uneven_fp16_storage():
    say("c4: uneven, FP16 storage")
    assert _uneven("c16") <= 1.0


def test_uneven_fp16_schedules_agree():
    """FP16 storage on the uneven plan: every schedule (persistent, one
    workgroup per tile, resident grid with the next tile's loads in flight)
    gives bit-identical forward and adjoint results."""
    say("c4 sizes, FP16 storage: every schedule")
    r, vals = workloads.make("c4")
    host = np.stack([vals.real, vals.imag], -1).astype(np.float16)
    t = torch.from_numpy(host).to(DEV).view(torch.complex32).reshape(-1)
    plan = qft.UnevenPlan(r.tolist(), qft.QFT_C16)
    names = plan.schedules
    assert any(n.endswith("/pipe") for n in names)
    fw, bw = [], []
    for i in range(len(names)):
        plan.schedule = i
        fw.append(plan.forward(t))
        bw.append(plan.adjoint(t))
    torch.cuda.synchronize()
    for i in range(1, len(names)):
        assert torch.equal(fw[i].view(torch.int16), fw[0].view(torch.int16)), names[i]
        assert torch.equal(bw[i].view(torch.int16), bw[0].view(torch.int16)), names[i]
    plan.close()


def test_c5_autograd_loss_gradient():
    say("c5: N=4096 B=512 loss = sum w |X|^2, autograd")
    x, w = workloads.make("c5")
    xt = torch.from_numpy(x).to(DEV).requires_grad_(True)
    wt = torch.from_numpy(w).to(DEV)
    X = qft.QFTFunction.apply(xt)
    loss = (wt * X.abs() ** 2).sum()
    loss.backward()
    g = xt.grad.cpu().numpy().astype(np.complex128)
    # analytic: for L = sum w |F x|^2, PyTorch's grad is 2 F^H (w * F x)
    x64 = x.astype(np.complex128)
    Xr = OB.cdft(x64)
    gref = 2 * np.conj(OB.cdft(np.conj(w * Xr)))
    rel, _ = check(g, gref, 2 * 12, what="c5 gradient")  # two transforms
    say(f"c5 grad rel-L2 {rel:.3e}")


def test_gradcheck_small_against_finite_differences():
    """N = 64, B = 8, seed 4: the GPU vector-Jacobian product against FP64
    central finite differences of the oracle (a linear map, so the FD are
    exact up to rounding); tolerance from the FP32 bound."""
    say("gradcheck N=64 B=8")
    rng = np.random.default_rng(4)
    N, B = 64, 8
    x = (rng.uniform(-1, 1, (B, N)) + 1j * rng.uniform(-1, 1, (B, N))).astype(np.complex64)
    v = (rng.uniform(-1, 1, (B, N)) + 1j * rng.uniform(-1, 1, (B, N))).astype(np.complex64)
    xt = torch.from_numpy(x).to(DEV).requires_grad_(True)
    X = qft.QFTFunction.apply(xt)
    # scalar L = Re <v, X>; grad wrt x (PyTorch convention) = F^H v
    L = (torch.from_numpy(v).to(DEV).conj() * X).real.sum()
    L.backward()
    g = xt.grad.cpu().numpy().astype(np.complex128)
    x64 = x.astype(np.complex128)
    h = 1e-3
    fd = np.zeros_like(x64)
    vv = v.astype(np.complex128)

    def Lf(z):
        return np.sum(np.real(np.conj(vv) * Q.qft(z)))

    for b in range(B):
        for n in range(N):
            for part, unit in ((0, 1.0), (1, 1j)):
                zp = x64.copy(); zp[b, n] += h * unit
                zm = x64.copy(); zm[b, n] -= h * unit
                d = (Lf(zp) - Lf(zm)) / (2 * h)
                fd[b, n] += d if part == 0 else 1j * d
    check(g, fd, 2 * 6, what="gradcheck")


def test_in_place_and_errors():
    say("in-place exec, alignment and overlap errors")
    x = workloads.uniform(55, (4, 512))
    t = torch.from_numpy(x).to(DEV)
    p = qft.Plan(9, 4)
    ref = p.forward(t).cpu().numpy()
    qft.qft_exec_fwd(p.handle, t.data_ptr(), t.data_ptr(), 0)  # in place
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), ref)
    L = _lib.lib()
    buf = torch.zeros(2 * 4 * 512 + 8, dtype=torch.complex64, device=DEV)
    base = buf.data_ptr()
    assert L.qft_exec_fwd(p.handle, base + 4, base + 4 * 512 * 8 * 2, None) == \
        _lib.QFT_ERROR_ALIGNMENT
    assert L.qft_exec_fwd(p.handle, base, base + 8 * 8, None) == _lib.QFT_ERROR_OVERLAP
    p.close()
    # multi-pass in place
    x = workloads.uniform(56, (2, 1 << 15))
    t = torch.from_numpy(x).to(DEV)
    p = qft.Plan(15, 2)
    ref = p.forward(t).cpu().numpy()
    qft.qft_exec_fwd(p.handle, t.data_ptr(), t.data_ptr(), 0)
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), ref)
    p.close()


def test_plan_info():
    p = qft.Plan(16, 256)
    info = p.info
    assert info["total_points"] == 256 * 65536
    assert info["algo_bytes"] == 2 * 256 * 65536 * 8
    assert info["flops_actual"] == 256 * (4 * 65536 * 16 - 6 * 65536 + 8)
    p.close()


@pytest.mark.parametrize("kind", ["uneven", "two_pass", "tile", "uneven_pipe", "tile_pipe",
                                  "tile_lds", "multi_pass_s13"])
def test_graph_capture_replays(kind):
    """exec neither allocates nor issues memsets, so it can be captured in a
    HIP graph (torch.cuda.CUDAGraph).  The graph is replayed several times with
    the program's own eager work and synchronisations in between, and every
    replay must equal the eager result bit for bit."""
    say(f"graph capture: {kind}")
    if kind.startswith("uneven"):
        r, vals = workloads.make("c4")
        x = torch.from_numpy(vals).to(DEV)
        plan = qft.UnevenPlan(r.tolist())
    elif kind == "two_pass":
        x = torch.from_numpy(workloads.normal(77, (8, 1 << 16))).to(DEV)
        plan = qft.Plan(16, 8)
    elif kind == "tile_pipe":
        x = torch.from_numpy(workloads.uniform(79, (600, 1 << 14))).to(DEV)
        plan = qft.Plan(14, 600)
    elif kind == "tile_lds":
        x = torch.from_numpy(workloads.uniform(80, (300, 1 << 12))).to(DEV)
        plan = qft.Plan(12, 300)
    elif kind == "multi_pass_s13":
        x = torch.from_numpy(workloads.normal(81, (2, 1 << 17))).to(DEV)
        plan = qft.Plan(17, 2)
    else:
        x = torch.from_numpy(workloads.uniform(78, (64, 1 << 10))).to(DEV)
        plan = qft.Plan(10, 64)
    # the schedule under test (the resident-grid, LDS-table or 2^13-segment one)
    suffix = {"uneven_pipe": "/pipe", "tile_pipe": "/pipe", "tile_lds": "/lds",
              "multi_pass_s13": "/s13"}.get(kind)
    if suffix:
        plan.schedule = next(i for i, n in enumerate(plan.schedules) if n.endswith(suffix))
    eager = plan.forward(x)
    torch.cuda.synchronize()
    out = torch.empty_like(x)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.forward(x, out)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        qft.qft_exec_fwd(plan.handle, x.data_ptr(), out.data_ptr(),
                         torch.cuda.current_stream().cuda_stream)
    for rep in range(4):
        out.zero_()
        junk = (x * (rep + 1)).sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {rep} differs"
        del junk
    plan.close()


@pytest.mark.parametrize("logn,B", [(5, 300), (10, 37), (12, 9), (13, 5), (14, 3)])
def test_uniform_and_uneven_kernels_agree(logn, B):
    """A batch of one size through a uniform plan (contiguous single-size
    kernel) and through an uneven plan (persistent kernel with an offset
    list, every schedule) gives bit-identical output: the same specialised
    body computes both."""
    say(f"uniform vs uneven kernel: N=2^{logn} B={B}")
    x = workloads.normal(4000 + logn, (B, 1 << logn))
    xt = torch.from_numpy(x).to(DEV)
    ref = qft.Plan(logn, B).forward(xt)
    up = qft.UnevenPlan([logn] * B)
    flat = xt.reshape(-1)
    for i in range(len(up.schedules)):
        up.schedule = i
        assert torch.equal(up.forward(flat).reshape(B, -1), ref), up.schedules[i]
    torch.cuda.synchronize()
    check(ref.cpu().numpy(), ref_fwd(x), logn, what="uniform vs uneven")
    up.close()


def test_uneven_schedules_and_autotune():
    """The uneven plan's schedules (one persistent launch for every size, or
    one launch per tile size; persistent, one workgroup per tile, or with
    the 2^14-point group on the resident grid that loads each next tile
    during the current one) agree bit for bit, the adjoint too; autotune
    times them all and keeps one."""
    say("schedules: uneven c4 sizes")
    r, vals = workloads.make("c4")
    xt = torch.from_numpy(vals).to(DEV)
    plan = qft.UnevenPlan(r.tolist())
    names = plan.schedules
    say(f"uneven schedules {names}")
    # 7 tile-size assignments (2^10 .. 2^14 tiles), each persistent and "/all",
    # and "/pipe" for the four whose 2^14 tiles form a group of their own
    # (455 tiles, more than the 256 resident workgroups)
    assert names[0] == "t14:6-14" and len(names) == 18
    assert "t10:6-10+t11:11+t12:12+t13:13+t14:14" in names
    pipes = [n for n in names if n.endswith("/pipe")]
    assert len(pipes) == 4 and "t13:6-13+t14:14/pipe" in pipes
    fw, bw = [], []
    for i in range(len(names)):
        plan.schedule = i
        fw.append(plan.forward(xt))
        bw.append(plan.adjoint(xt))
    torch.cuda.synchronize()
    for o in fw[1:]:
        assert torch.equal(o, fw[0])
    for o in bw[1:]:
        assert torch.equal(o, bw[0])
    times = plan.autotune(xt, reps=3)
    say(f"autotune ms {times}")
    assert set(times) == set(names) and all(t > 0 for t in times.values())
    assert plan.schedules[plan.schedule] == min(times, key=times.get)
    assert torch.equal(plan.forward(xt), fw[0])
    with pytest.raises(qft.QFTError):
        plan.schedule = len(names)
    plan.close()


def _rdft_ref(x):
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[-1]
    re, im = Q.rdft(x, N, Q.Ops())
    ref = re.astype(np.complex128)
    if N > 2:
        ref[..., 1:N // 2] += 1j * im
    return ref


@pytest.mark.parametrize("logn", range(1, 15))
def test_rdft_all_tile_sizes(logn):
    """Real-input transform (rdft, Sec. 4.2): half spectrum against the
    oracle's rdft, with an odd number of signals (the last slot's second lane
    empty)."""
    N = 1 << logn
    B = 7 if logn > 10 else 33
    say(f"rdft: N=2^{logn} B={B}")
    x = np.ascontiguousarray(workloads.normal(5000 + logn, (B, N)).real.astype(np.float32))
    H = qft.rdft(torch.from_numpy(x).to(DEV))
    torch.cuda.synchronize()
    assert H.shape == (B, N // 2 + 1) and H.dtype == torch.complex64
    check(H.cpu().numpy(), _rdft_ref(x), logn, what=f"rdft 2^{logn}")


def test_rdft_matches_complex_path_and_fp16():
    """The rdft of x equals the first N/2+1 bins of the complex transform of
    x + 0i; FP16 storage within the output-rounding bound."""
    say("rdft vs complex, fp16")
    logn, B = 12, 64
    x = np.ascontiguousarray(workloads.uniform(6000, (B, 1 << logn)).real.astype(np.float32))
    xt = torch.from_numpy(x).to(DEV)
    H = qft.rdft(xt)
    X = qft.fft(xt.to(torch.complex64))
    torch.cuda.synchronize()
    h = H.cpu().numpy().astype(np.complex128)
    full = X.cpu().numpy().astype(np.complex128)[:, :(1 << logn) // 2 + 1]
    check(h, full, 2 * logn, what="rdft vs complex")  # both sides carry FP32 error
    H16 = qft.rdft(xt.half())
    torch.cuda.synchronize()
    h16 = H16.view(torch.float16).reshape(B, -1, 2).float().cpu().numpy()
    ref16 = _rdft_ref(x.astype(np.float16).astype(np.float64))
    check(h16[..., 0] + 1j * h16[..., 1], ref16, logn, fp16=True, what="rdft fp16")


@pytest.mark.parametrize("logn", [1, 2, 3, 6, 10, 13, 14])
def test_dct0_dst0(logn):
    """Standalone DCT-0 / DST-0 (dct on s_dc_tt, dst on s_ds_tt) against the
    oracle, together, alone, and in place."""
    N = 1 << logn
    h = N // 2
    B = 5
    say(f"dct0/dst0: N=2^{logn} B={B}")
    c = np.ascontiguousarray(workloads.uniform(7000 + logn, (B, h + 1)).real.astype(np.float32))
    d = np.ascontiguousarray(workloads.uniform(7100 + logn, (B, max(h - 1, 1))).real
                             .astype(np.float32)[:, :h - 1])
    refC = Q.dct(c.astype(np.float64), N, Q.Ops())
    ct, dt_ = torch.from_numpy(c).to(DEV), torch.from_numpy(d.copy()).to(DEV)
    plan = qft.RealPlan(logn, B)
    C, S = plan.dct0_dst0(ct, dt_ if h > 1 else None)
    C1 = qft.dct0(ct)
    torch.cuda.synchronize()
    check(C.cpu().numpy(), refC, logn, what="dct0")
    assert torch.equal(C, C1)
    if h > 1:
        refS = Q.dst(d.astype(np.float64), N, Q.Ops())
        if h > 2:
            check(S.cpu().numpy(), refS, logn, what="dst0")
        else:  # one value, S(1) = d(1): an exact copy
            assert np.array_equal(S.cpu().numpy().astype(np.float64), refS)
        assert torch.equal(qft.dst0(dt_), S)
        # in place: c -> C and d -> S in the input buffers
        qft.qft_exec_dct0_dst0(plan.handle, ct.data_ptr(), dt_.data_ptr(), ct.data_ptr(),
                               dt_.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        assert torch.equal(ct, C) and torch.equal(dt_, S)
    plan.close()


def test_real_plan_errors():
    say("real plan error codes")
    plan = qft.RealPlan(10, 4)
    x = torch.zeros(4, 1024, device=DEV)
    y = torch.zeros(4, 1024, dtype=torch.complex64, device=DEV)
    with pytest.raises(qft.QFTError):  # complex exec on a real plan
        qft.qft_exec_fwd(plan.handle, y.data_ptr(), y.data_ptr(), 0)
    with pytest.raises(qft.QFTError):  # overlapping rdft buffers
        qft.qft_exec_rdft(plan.handle, x.data_ptr(), x.data_ptr() + 64, 0)
    with pytest.raises(qft.QFTError):  # a half-given pair
        qft.qft_exec_dct0_dst0(plan.handle, x.data_ptr(), None, None, None, 0)
    cplan = qft.Plan(10, 4)
    with pytest.raises(qft.QFTError):  # rdft on a complex plan
        qft.qft_exec_rdft(cplan.handle, x.data_ptr(), y.data_ptr(), 0)
    plan.close()
    cplan.close()


@pytest.mark.parametrize("logn,B", [(15, 3), (16, 4), (18, 1)])
def test_real_input_multipass_sizes(logn, B):
    """Real-input plans beyond a tile: the multi-pass path on transform slots
    of two real signals, rdft, DCT-0 and DST-0 against the oracle (the C copy
    of the recursion for the DCT-0/DST-0 of every size)."""
    N, h = 1 << logn, 1 << (logn - 1)
    say(f"real multi-pass: N=2^{logn} B={B}")
    x = np.ascontiguousarray(workloads.normal(8000 + logn, (B, N)).real.astype(np.float32))
    H = qft.rdft(torch.from_numpy(x).to(DEV))
    torch.cuda.synchronize()
    ref = OB.cdft(x.astype(np.complex128))[:, :h + 1]
    check(H.cpu().numpy(), ref, logn, what=f"rdft 2^{logn}")
    c = np.ascontiguousarray(workloads.uniform(8100 + logn, (B, h + 1)).real.astype(np.float32))
    d = np.ascontiguousarray(workloads.uniform(8200 + logn, (B, h - 1)).real.astype(np.float32))
    C = qft.dct0(torch.from_numpy(c).to(DEV))
    S = qft.dst0(torch.from_numpy(d).to(DEV))
    torch.cuda.synchronize()
    check(C.cpu().numpy(), OB.dct(c.astype(np.float64), N), logn, what=f"dct0 2^{logn}")
    check(S.cpu().numpy(), OB.dst(d.astype(np.float64), N), logn, what=f"dst0 2^{logn}")


def test_broadband_2p24():
    """One N = 2^24 transform of N(0,1) samples: every bin carries a
    comparable share of the energy, so the per-bin bound checks all 16.7 M
    bins of the multi-pass path (the tones of c3 leave most bins near the
    noise floor)."""
    say("broadband: N=2^24 B=1 N(0,1) seed 24")
    x = workloads.normal(24, (1, 1 << 24))
    X = gpu_fwd(x)
    rel, worst = check(X, OB.cdft(x.astype(np.complex128)), 24, what="broadband 2^24")
    say(f"broadband 2^24 rel-L2 {rel:.3e}, worst bin {worst:.2f} of its bound")


def test_uneven_with_long_transforms():
    """An uneven plan whose transforms beyond a tile (2^15 and 2^16 two-pass,
    2^17 multi-pass) sit at nonzero offsets between tile-sized ones, in every
    schedule, forward and adjoint."""
    sizes = [6, 12, 15, 16, 17, 6, 15, 9, 16]
    say(f"uneven with long transforms: {sizes}")
    off = np.concatenate([[0], np.cumsum([1 << s for s in sizes])])
    vals = workloads.normal(4321, (int(off[-1]),))
    plan = qft.UnevenPlan(sizes)
    xt = torch.from_numpy(vals).to(DEV)
    outs = []
    for i in range(len(plan.schedules)):
        plan.schedule = i
        outs.append((plan.forward(xt), plan.adjoint(xt)))
    torch.cuda.synchronize()
    for f, b in outs[1:]:
        assert torch.equal(f, outs[0][0]) and torch.equal(b, outs[0][1])
    got_f = outs[0][0].cpu().numpy()
    got_b = outs[0][1].cpu().numpy()
    for i, lg in enumerate(sizes):
        seg = vals[off[i]:off[i + 1]].astype(np.complex128)[None]
        check(got_f[off[i]:off[i + 1]][None], OB.cdft(seg), lg, what=f"uneven #{i} 2^{lg}")
        check(got_b[off[i]:off[i + 1]][None], np.conj(OB.cdft(np.conj(seg))), lg,
              what=f"uneven adjoint #{i} 2^{lg}")
    plan.close()


@pytest.mark.parametrize("logn,B", [(12, 1500), (13, 700), (14, 300), (16, 70), (17, 6)])
@pytest.mark.parametrize("c16", [False, True])
def test_schedules_agree_adjoint_and_fp16(logn, B, c16):
    """Every schedule of a uniform plan (table in global memory or LDS,
    resident grids, two-pass grids, multi-pass splits and segment sizes)
    gives bit-identical results for the adjoint too, and with FP16 storage
    in both directions; the first schedule's results match the oracle."""
    say(f"schedules agree: N=2^{logn} B={B} fp16={c16}")
    x = workloads.uniform(9300 + logn, (B, 1 << logn)).astype(np.complex64)
    if c16:
        host = np.stack([x.real, x.imag], -1).astype(np.float16)
        xin = host[..., 0].astype(np.float64) + 1j * host[..., 1].astype(np.float64)
        t = torch.from_numpy(host).to(DEV).view(torch.complex32).reshape(B, -1)
        p = qft.Plan(logn, B, qft.QFT_C16)
    else:
        xin = x.astype(np.complex128)
        t = torch.from_numpy(x).to(DEV)
        p = qft.Plan(logn, B)
    names = p.schedules
    assert len(names) > 1
    outs = []
    for i in range(len(names)):
        p.schedule = i
        outs.append((p.forward(t), p.adjoint(t)))
    torch.cuda.synchronize()
    for i, (f, b) in enumerate(outs[1:], 1):
        assert torch.equal(f, outs[0][0]), names[i]
        assert torch.equal(b, outs[0][1]), names[i]

    def host_of(y):
        if not c16:
            return y.cpu().numpy().astype(np.complex128)
        o = y.view(torch.float16).reshape(B, -1, 2).float().cpu().numpy().astype(np.float64)
        return o[..., 0] + 1j * o[..., 1]

    check(host_of(outs[0][0]), ref_fwd(xin), logn, fp16=c16, what=f"2^{logn} schedules fwd")
    check(host_of(outs[0][1]), np.conj(ref_fwd(np.conj(xin))), logn, fp16=c16,
          what=f"2^{logn} schedules adjoint")
    p.close()


def test_uneven_runs_of_long_transforms():
    """Runs of same-size long transforms that lie back to back (2^15, 2^16,
    2^17; the 2^16 run longer than one batched launch holds, 2^22 cells)
    run as batched execs: every transform matches the oracle, forward and
    adjoint."""
    sizes = [15, 15, 15, 16, 16, 12] + [16] * 66 + [17, 17, 9, 15]
    say(f"uneven runs of long transforms: {len(sizes)} transforms")
    off = np.concatenate([[0], np.cumsum([1 << s for s in sizes])])
    vals = workloads.normal(4322, (int(off[-1]),))
    plan = qft.UnevenPlan(sizes)
    xt = torch.from_numpy(vals).to(DEV)
    got_f = plan.forward(xt).cpu().numpy()
    got_b = plan.adjoint(xt).cpu().numpy()
    for i, lg in enumerate(sizes):
        seg = vals[off[i]:off[i + 1]].astype(np.complex128)[None]
        check(got_f[off[i]:off[i + 1]][None], OB.cdft(seg), lg, what=f"run #{i} 2^{lg}")
        check(got_b[off[i]:off[i + 1]][None], np.conj(OB.cdft(np.conj(seg))), lg,
              what=f"run adjoint #{i} 2^{lg}")
    plan.close()


def test_two_streams_share_no_scratch():
    """fft() on two streams at once with the same shape (N = 2^16, a plan
    with scratch memory): each stream gets a plan of its own, and both results
    match the oracle."""
    say("two streams, N=2^16 B=16")
    xa = workloads.normal(61, (16, 1 << 16))
    xb = workloads.normal(62, (16, 1 << 16))
    ta, tb = torch.from_numpy(xa).to(DEV), torch.from_numpy(xb).to(DEV)
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    outs = {}
    for _ in range(3):
        with torch.cuda.stream(sa):
            outs["a"] = qft.fft(ta)
        with torch.cuda.stream(sb):
            outs["b"] = qft.fft(tb)
    torch.cuda.synchronize()
    check(outs["a"].cpu().numpy(), OB.cdft(xa.astype(np.complex128)), 16, what="stream a")
    check(outs["b"].cpu().numpy(), OB.cdft(xb.astype(np.complex128)), 16, what="stream b")


@pytest.mark.parametrize("logn,B", [(18, 2), (12, 64), (12, 1500), (14, 300), (9, 9000),
                                    (15, 300), (16, 260)])
def test_stage_schedules_agree_and_autotune_is_cached(logn, B, tmp_path, monkeypatch):
    """A uniform plan's schedules (multi-pass: splits of the global passes;
    tile sizes: the specialised kernel, one workgroup per tile and, where
    there are more tiles than resident workgroups, on a resident grid that
    loads each next tile during the current one, and the size-generic
    persistent kernel with each tile size; two-pass: pass A as a persistent
    grid, at these batches smaller than the tile count, and one workgroup
    per tile) give
    bit-identical results; autotune keeps the
    fastest and records it in the schedule cache, and a new plan of the same
    shape starts on the cached schedule (also one written by hand)."""
    cache = tmp_path / "schedules.json"
    monkeypatch.setenv("QFT_SCHEDULE_CACHE", str(cache))
    say(f"stage schedules: N=2^{logn} B={B}")
    x = torch.from_numpy(workloads.normal(5100 + logn, (B, 1 << logn))).to(DEV)
    p = qft.Plan(logn, B)
    names = p.schedules
    say(f"schedules {names}")
    assert len(names) > 1 and p.schedule == 0
    outs = []
    for i in range(len(names)):
        p.schedule = i
        outs.append(p.forward(x))
    torch.cuda.synchronize()
    for i, o in enumerate(outs[1:], 1):
        assert torch.equal(o, outs[0]), names[i]
    check(outs[0].cpu().numpy(), ref_fwd(x.cpu().numpy()), logn, what=f"2^{logn} schedules")
    times = p.autotune(x, reps=2)
    best = names[p.schedule]
    assert best == min(times, key=times.get)
    doc = json.load(open(cache))
    assert best in doc["entries"].values()
    p2 = qft.Plan(logn, B)
    assert p2.schedules[p2.schedule] == best
    # a hand-written entry naming another schedule is followed
    key = [k for k, v in doc["entries"].items() if v == best][0]
    other = names[-1] if best != names[-1] else names[0]
    doc["entries"][key] = other
    json.dump(doc, open(cache, "w"))
    p3 = qft.Plan(logn, B)
    assert p3.schedules[p3.schedule] == other
    assert torch.equal(p3.forward(x), outs[0])
    # an entry naming no schedule of the plan is ignored
    doc["entries"][key] = "no-such-schedule"
    json.dump(doc, open(cache, "w"))
    assert qft.Plan(logn, B).schedule == 0
    for q in (p, p2, p3):
        q.close()


def _fixed_ref(x):
    from oracle import qft_fixed as F
    return F.cdft_fixed(x)


@pytest.mark.parametrize("logn,B", [(1, 3), (2, 3), (3, 3), (4, 5), (5, 4), (6, 3), (7, 3),
                                    (8, 3), (9, 3), (10, 3), (11, 2), (12, 3), (13, 2),
                                    (14, 2), (15, 2), (16, 2),
                                    (2, 2100), (4, 600), (8, 37), (11, 5)])
def test_fixed_point_bit_exact(logn, B):
    """Fixed point (QFT_I32): forward and adjoint bit-identical to the integer
    oracle, on inputs within the overflow-free range and on full-range int32
    inputs (wrapping); in range, close to the exact DFT.  Small transforms
    share a workgroup (2^12 / N of them, each with its own threads): the
    batches with several workgroups and a partly filled last one check
    that."""
    N = 1 << logn
    say(f"fixed point: N=2^{logn} B={B}")
    rng = np.random.default_rng(3300 + logn)
    plan = qft.FixedPlan(logn, B)
    for lim in (1 << (28 - logn), 1 << 31):
        x = rng.integers(-lim, lim, (B, N, 2)).astype(np.int32)
        xt = torch.from_numpy(x).to(DEV)
        X = plan.forward(xt).cpu().numpy().astype(np.int64)
        assert np.array_equal(X, _fixed_ref(x)), lim
        Y = plan.adjoint(xt).cpu().numpy().astype(np.int64)
        assert np.array_equal(Y, _fixed_ref(x[..., ::-1])[..., ::-1]), lim
        if lim < (1 << 31):
            exact = OB.cdft((x[..., 0] + 1j * x[..., 1]).astype(np.complex128))
            err = D.relative_l2(X[..., 0] + 1j * X[..., 1], exact).max()
            assert err < 1e-3, err
    plan.close()
