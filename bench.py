"""Benchmark: exact modular matrix multiplication on one MI355X.

Workload: m = n = k = 4096, p = 8388593 (largest prime below 2^23),
alpha = 3, beta = 5, A, B, C seeded uniform residues resident in HBM.
One step = one ff_fgemm call on the INT8 path with 4 signed 7-bit digits:
slicing of A and B into digit planes, 16 digit-pair products on INT8 matrix
cores with int32 sums, and the epilogue that recombines the digits modulo p
and applies alpha and beta.  The metric is 2mnk / t (Gop/s); the same
workload is also timed on the FP64 matrix-core path (K-block 512) and with
8-bit digits (3 slices).

The JSON line carries the roofline of the dominant kernel (the INT8 digit
GEMM, measured with HIP events around its launches) and the CPU oracle timed
on a bounded sample of the same product on the host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_INT8_TOPS = 5000.0   # MI355X dense INT8 matrix peak, TOP/s
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 matrix peak, TFLOP/s

M = N = K = 4096
P = 8388593
ALPHA, BETA = 3, 5


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target length of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    return ap.parse_args()


def time_path(ff, torch, dA, dB, dC, opts, steps, warmup):
    """Returns (ms per step, per-step ms list, profile dict)."""
    for _ in range(warmup):
        ff.fgemm(P, dA, dB, dC, ALPHA, BETA, opts=opts)
    torch.cuda.synchronize()
    ff.ff_profile_enable(1)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(steps):
        ff.fgemm(P, dA, dB, dC, ALPHA, BETA, opts=opts)
        ev[i + 1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    prof = ff.ff_profile_read()
    ff.ff_profile_enable(0)
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return wall / steps, per, prof


def cpu_baseline(A, B, C, seconds):
    """The oracle on a bounded sample: full rows of C = 3AB + 5C mod p."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    os.environ.setdefault("OMP_NUM_THREADS", str(threads))
    # calibration on 4 rows, then enough rows for about `seconds`
    t = time.perf_counter()
    oracle.fgemm(P, A[:4], B, C[:4], ALPHA, BETA)
    dt = max(time.perf_counter() - t, 1e-3)
    rows = int(max(4, min(M, 4 * seconds / dt)))
    t = time.perf_counter()
    oracle.fgemm(P, A[:rows], B, C[:rows], ALPHA, BETA)
    dt = time.perf_counter() - t
    return {"value": 2.0 * rows * N * K / dt / 1e9, "unit": "Gop/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{rows} full rows of the 4096 x 4096 product ({rows * N * K:.3g} "
                      f"multiply-adds, {dt:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_cs_0601133_amd import ffgemm as ff
    from paper_cs_0601133_amd import synth

    torch.cuda.set_device(0)
    ff.ff_init()
    A = synth.residues(synth.seed_for(2, 1), (M, K), P)
    B = synth.residues(synth.seed_for(2, 2), (K, N), P)
    C = synth.residues(synth.seed_for(2, 3), (M, N), P)
    dA = torch.from_numpy(A.view(np.int32)).cuda()
    dB = torch.from_numpy(B.view(np.int32)).cuda()
    dC = torch.from_numpy(C.view(np.int32)).cuda()

    ops = 2.0 * M * N * K
    res = {}
    for name, opts in (("int8_d7", ff.make_opts(path=ff.FF_PATH_INT8, digit_bits=7,
                                                 winograd_levels=0)),
                       ("int8_d8", ff.make_opts(path=ff.FF_PATH_INT8, digit_bits=8,
                                                 winograd_levels=0)),
                       ("fp64", ff.make_opts(path=ff.FF_PATH_FP64, winograd_levels=0))):
        info = ff.ff_plan_query(P, 0, 0, M, N, K, opts)
        ms, per, prof = time_path(ff, torch, dA, dB, dC, opts, args.steps, args.warmup)
        gemm_ms = prof["gemm_ms"] / max(prof["gemm_launches"], 1)
        slice_ms = prof["slice_ms"] / max(prof["slice_launches"], 1)
        per_sorted = sorted(per)
        r = {"ms_per_step": ms, "gops": ops / ms / 1e6,
             "p50_ms": float(np.percentile(per_sorted, 50)),
             "p99_ms": float(np.percentile(per_sorted, 99)),
             "gemm_kernel_ms": gemm_ms, "slice_kernel_ms": slice_ms,
             "slices": info.slices, "kblock": info.kblock}
        if info.path == ff.FF_PATH_INT8:
            mfma_ops = info.slices ** 2 * ops
            r["mfma_tops"] = mfma_ops / gemm_ms / 1e9
            r["frac_int8_peak"] = r["mfma_tops"] / PEAK_INT8_TOPS
        else:
            r["mfma_tflops"] = ops / gemm_ms / 1e9
            r["frac_fp64_peak"] = r["mfma_tflops"] / PEAK_FP64_TFLOPS
        r["effective_frac_fp64_peak"] = ops / ms / 1e9 / PEAK_FP64_TFLOPS
        res[name] = r

    head = res["int8_d7"]
    line = {
        "metric": "modular GEMM Gop/s (2mnk/t, bit-exact) INT8-sliced vs FP64; p50/p99 latency",
        "value": head["gops"],
        "unit": "Gop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": "fgemm m=n=k=4096, p=8388593, alpha=3, beta=5; INT8 path, "
                               "4 signed 7-bit digit slices",
                   "m": M, "n": N, "k": K, "p": P, "alpha": ALPHA, "beta": BETA},
        "p50_ms": head["p50_ms"],
        "p99_ms": head["p99_ms"],
        "roofline": {"bound": "mfma", "achieved": head["mfma_tops"],
                     "peak": PEAK_INT8_TOPS, "unit": "TOP/s",
                     "frac": head["frac_int8_peak"], "traffic": None,
                     "kernel": "k_fgemm_i8<S=4>",
                     "ops_per_launch": 16 * ops},
        "paths": res,
        "int8_vs_fp64_speedup": res["fp64"]["ms_per_step"] / head["ms_per_step"],
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(A, B, C, args.cpu_seconds)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
