"""The allocation-free entry point qft_exec_fwd_static (static scratch per GPU)
against the plan-based qft_exec_fwd on the same inputs, to the parity bar of
tests/parity.py, on consecutive calls of decreasing size (the scratch keeps
the previous call's contents), in both storage types, and replayed from a
captured HIP graph."""
import sys

import numpy as np
import pytest

import workloads
from tests.parity import check

torch = pytest.importorskip("torch")
import paper_1301_0763_amd as qft  # noqa: E402
from paper_1301_0763_amd import _lib  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def _static(x, log2n, dtype=qft.QFT_C32):
    out = torch.empty_like(x)
    qft.qft_exec_fwd_static(log2n, x.numel() >> log2n, dtype, x.data_ptr(), out.data_ptr(),
                            torch.cuda.current_stream().cuda_stream)
    return out


def _planned(x, log2n, dtype=qft.QFT_C32):
    p = qft.Plan(log2n, x.numel() >> log2n, dtype)
    y = p.forward(x)
    torch.cuda.synchronize()
    p.close()
    return y


def test_static_matches_plan_on_consecutive_calls():
    # largest first (the two-pass heap nearly fills the scratch), then smaller
    cases = [(16, 120, 71), (15, 9, 72), (12, 33, 73), (16, 2, 74), (5, 3, 75)]
    for log2n, B, seed in cases:
        say(f"static vs plan: N=2^{log2n} B={B}")
        x = torch.from_numpy(workloads.normal(seed, (B, 1 << log2n))).to(DEV)
        got = _static(x, log2n)
        ref = _planned(x, log2n)
        torch.cuda.synchronize()
        same = torch.equal(got, ref)
        say(f"  bit-identical to the plan: {same}")
        check(got.cpu().numpy(), ref.cpu().numpy(), log2n, what=f"static 2^{log2n} x {B}")
        # same kernels, and the constant table computed on the device in FP64
        # rounds to the host table's FP32 values, so the results are identical
        assert same


def test_static_fp16_storage():
    for log2n, B, seed in [(16, 40, 81), (13, 5, 82)]:
        say(f"static fp16: N=2^{log2n} B={B}")
        x = workloads.uniform(seed, (B, 1 << log2n)).astype(np.complex64)
        host = np.stack([x.real, x.imag], -1).astype(np.float16)
        t = torch.from_numpy(host).to(DEV).view(torch.complex32).reshape(B, -1)
        got = _static(t, log2n, qft.QFT_C16)
        ref = _planned(t, log2n, qft.QFT_C16)
        torch.cuda.synchronize()
        g = got.view(torch.float16).reshape(B, -1, 2).float().cpu().numpy()
        r = ref.view(torch.float16).reshape(B, -1, 2).float().cpu().numpy()
        check(g[..., 0] + 1j * g[..., 1], r[..., 0] + 1j * r[..., 1], log2n, fp16=True,
              what=f"static fp16 2^{log2n}")


def test_static_rejects_beyond_scratch():
    x = torch.zeros(128, 1 << 16, dtype=torch.complex64, device=DEV)
    with pytest.raises(qft.QFTError) as e:
        _static(x, 16)
    assert e.value.status == _lib.QFT_ERROR_SCRATCH


def test_static_graph_replay():
    log2n, B = 16, 16
    x = torch.from_numpy(workloads.normal(91, (B, 1 << log2n))).to(DEV)
    eager = _static(x, log2n)
    torch.cuda.synchronize()
    out = torch.empty_like(x)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        qft.qft_exec_fwd_static(log2n, B, qft.QFT_C32, x.data_ptr(), out.data_ptr(),
                                s.cuda_stream)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        qft.qft_exec_fwd_static(log2n, B, qft.QFT_C32, x.data_ptr(), out.data_ptr(),
                                torch.cuda.current_stream().cuda_stream)
    for rep in range(3):
        out.zero_()
        _static(x[:4].contiguous(), log2n)  # other work on the same scratch between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {rep}"
