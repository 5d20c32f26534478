"""Benchmark of the improved-QFT forward transform on one MI355X.

Workload: batched forward complex FP32 DFT, N = 2^16, batch 256, re/im
i.i.d. N(0, 1) from seed 1 (synthetic; the paper has no dataset).  A step is
one qft_exec_fwd over the whole batch (every step of the transform: fold,
forward rounds, backward rounds, DCT-0/DST-0 chain, combine), with input and
output resident in HBM.

Prints one JSON line: throughput in GFLOP/s at the 5 N log2 N convention,
the HBM roofline of the timed kernels (algorithmic bytes 16 N per transform:
read 8N + write 8N, over HIP-event time on the launch stream), the FP64 CPU
oracle timed on this host as a baseline, and the error against that oracle.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "batched complex FFT GFLOP/s (5N log2N) + HBM GB/s % roofline; fwd+bwd speedup"
HBM_PEAK_GBS = 8000.0


def cpu_baseline(x, log2n):
    """FP64 C oracle (OpenMP over the batch) on this host's cores."""
    from oracle import build as OB
    lib = OB.load()
    threads = lib.qft_ref_threads()
    x64 = np.ascontiguousarray(x.astype(np.complex128))
    N = 1 << log2n
    B = x64.shape[0]
    t0 = time.perf_counter()
    X = OB.cdft(x64)
    dt = time.perf_counter() - t0
    gflops = 5.0 * N * log2n * B / dt / 1e9
    return X, dict(value=round(gflops, 3), unit="GFLOP/s", cores=threads, kind="oracle",
                   sample=f"the full batch ({B} transforms of N=2^{log2n}), FP64 recursive "
                          f"improved QFT in C, one pass, {dt:.2f} s wall")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--log2n", type=int, default=16)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--calib-copy", action="store_true",
                    help="time a plain device copy of the same bytes instead (for counter "
                         "calibration and the practical bandwidth ceiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the transform batch is not sharded across "
              "GPUs in this build (see the design notes); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1301_0763_amd as qft
    import workloads

    log2n, B = args.log2n, args.batch
    N = 1 << log2n
    dev = torch.device("cuda:0")
    if log2n == 16 and B == 256:
        x = workloads.make("c2")
        wname = "c2"
    else:
        x = workloads.normal(1, (B, N))
        wname = "custom"
    xt = torch.from_numpy(x).to(dev)
    yt = torch.empty_like(xt)
    plan = qft.Plan(log2n, B)
    stream = torch.cuda.current_stream(dev)
    sp = stream.cuda_stream

    def step():
        if args.calib_copy:
            yt.copy_(xt)
        else:
            qft.qft_exec_fwd(plan.handle, xt.data_ptr(), yt.data_ptr(), sp)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps

    info = plan.info
    if args.calib_copy:
        nbytes = 2 * xt.numel() * xt.element_size()
        print(json.dumps({"calibration": "device copy", "bytes_moved": nbytes,
                          "ms": round(ms, 5), "GB/s": round(nbytes / (ms * 1e-3) / 1e9, 1)}))
        return
    flop5 = info["flops_5nlogn"]
    gflops = flop5 / (ms * 1e-3) / 1e9
    algo_bytes = info["algo_bytes"]
    achieved = algo_bytes / (ms * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{wname}: batched forward complex FP32 DFT, N=2^{log2n}, batch {B}, "
                        "re/im N(0,1) seed 1",
            "log2n": log2n, "batch": B, "storage": "complex64",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "qft_exec_fwd, all launches of one step",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
        },
        "actual_flops_gflops": round(info["flops_actual"] / (ms * 1e-3) / 1e9, 2),
        "wall_s_timed_region": round(wall, 4),
    }

    # accuracy of this run against the FP64 oracle (first 8 transforms) and
    # the CPU baseline over the whole batch
    Y = yt.cpu().numpy()
    if not args.no_cpu:
        Xref, cb = cpu_baseline(x, log2n)
        out["cpu_baseline"] = cb
        from oracle import direct as D
        err = D.relative_l2(Y, Xref)
        out["error_vs_fp64_oracle"] = {"rel_l2_mean": float(f"{err.mean():.3e}"),
                                       "rel_l2_max": float(f"{err.max():.3e}"),
                                       "target": 1e-5 * log2n}
    print(json.dumps(out))
    plan.close()


if __name__ == "__main__":
    main()
