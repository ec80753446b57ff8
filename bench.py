"""Benchmark: exact modular matrix multiplication on one MI355X.

Headline workload (the metric's configuration): m = n = k = 4096,
p = 8388593 (largest prime below 2^23), alpha = 3, beta = 5, A, B, C seeded
uniform residues resident in HBM.  One step = one ff_fgemm call on the INT8
path with 4 signed 7-bit digits: slicing of A and B into digit planes, 16
digit-pair products on INT8 matrix cores with int32 sums, and the epilogue
that recombines the digits modulo p and applies alpha and beta.  The metric
is 2mnk / t (Gop/s); the same workload is also timed on the FP64
matrix-core path (operands packed as centered doubles, reduction every 512
products), with 8-bit digits (3 slices), and with one Winograd level on the
7-bit path (reported beside the plain product as effective 2mnk / t, never
as the headline value).

The JSON line also carries the roofline of the dominant kernel (the INT8
digit GEMM, timed with HIP events around its launches), the CPU oracle timed
on a bounded sample of the same product, and the other workloads: the
n = 256 latency case, n = 8192 at p = 251 and with Winograd levels, the
64-job multi-modular batch (plain, persistent and graph-replayed), the
triangular solve with matrix right-hand side (Section 4), the LQUP
factorisation (Section 5.1), the symmetric product A D A^T (Section 6) and
the Poisson serving stream.
"""
import argparse
import ctypes
import hashlib
import json
import math
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_fgemm_i8_S4_n4096_traffic.txt")
# sources the INT8 digit GEMM is compiled from (the traffic figures hold
# only while these are unchanged)
I8_SOURCES = [os.path.join(ROOT, "paper_cs_0601133_amd", "csrc", f)
              for f in ("kernels_i8.hip", "ff_ring.h", "ff_device.h")]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--settle-s", type=float, default=0.3,
                    help="untimed calls of each timed workload for this long before its "
                         "warm-up steps: the GPU's clocks take tens of ms of sustained "
                         "matrix-core load to settle")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="target length of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="time only the 4096^3 workload (profiler runs)")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--ftrsm-only", action="store_true",
                    help="time only the triangular solves (profiler runs)")
    ap.add_argument("--aat-only", action="store_true",
                    help="time only the symmetric product (profiler runs)")
    ap.add_argument("--lqup-only", action="store_true",
                    help="time only the LQUP factorisations (profiler runs)")
    ap.add_argument("--n8192-only", action="store_true",
                    help="time only the 8192^3 products with 0-2 Winograd levels (profiler runs)")
    ap.add_argument("--latency-only", action="store_true",
                    help="time only the 256^3 latency workload (profiler runs)")
    ap.add_argument("--multimodular-only", action="store_true",
                    help="time only the 64-job multi-modular batch (profiler runs)")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the Poisson serving stream (profiler runs)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gops(ops, ms):
    return ops / ms / 1e6


SETTLE_S = 0.3


def settle(torch, fn, seconds=None):
    """Untimed calls for about `seconds` of wall time (the clock controller
    needs tens of ms of sustained load to reach its steady state)."""
    seconds = SETTLE_S if seconds is None else seconds
    t0 = time.perf_counter()
    calls = 0
    while time.perf_counter() - t0 < seconds:
        fn()
        calls += 1
        if calls % 8 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    return calls


def time_calls(torch, fn, steps, warmup, ff=None):
    """Per-call event timing on torch's stream; returns (mean ms, per-call
    ms, profile of the library's kernels).  The timed calls bracket only the
    matrix-core kernel with HIP events (its duration gives the roofline); the
    operand passes (slicing, packing) are timed on a few extra calls after
    the timed region, so that their events do not lengthen the timed steps.
    Before the warm-up steps, untimed calls run for SETTLE_S seconds."""
    settle(torch, fn)
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if ff:
        ff.ff_profile_enable(ff.FF_PROFILE_GEMM)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(steps):
        fn()
        ev[i + 1].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    prof = None
    if ff:
        prof = ff.ff_profile_read()
        ff.ff_profile_enable(ff.FF_PROFILE_PREP)
        for _ in range(min(steps, 5)):
            fn()
        prep = ff.ff_profile_read()
        ff.ff_profile_enable(0)
        prof["slice_ms"], prof["slice_launches"] = prep["slice_ms"], prep["slice_launches"]
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return wall / steps, per, prof


def summarize(per):
    return {"p50_ms": float(np.percentile(per, 50)), "p99_ms": float(np.percentile(per, 99))}


def residues_dev(torch, shape, p, seed):
    from paper_cs_0601133_amd import synth
    a = synth.residues(seed, shape, p)
    return torch.from_numpy(a.view(np.int32)).cuda(), a


def cpu_baseline(A, B, C, seconds, gpu_rows=None):
    """The oracle on a bounded sample: full rows of C = 3AB + 5C mod p.  The
    rows are also compared with the same rows of one GPU call (gpu_rows)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    os.environ.setdefault("OMP_NUM_THREADS", str(threads))
    # probe with one row per thread (the oracle parallelises over rows), then
    # size the sample to about `seconds` of work in whole rounds of rows
    probe = max(4, threads)
    t = time.perf_counter()
    oracle.fgemm(P, A[:probe], B, C[:probe], ALPHA, BETA)
    dt = max(time.perf_counter() - t, 1e-3)
    rows = int(max(probe, min(M, probe * max(1, round(seconds / dt)))))
    t = time.perf_counter()
    want = oracle.fgemm(P, A[:rows], B, C[:rows], ALPHA, BETA)
    dt = time.perf_counter() - t
    match = None if gpu_rows is None else bool(np.array_equal(want, gpu_rows[:rows]))
    return {"value": 2.0 * rows * N * K / dt / 1e9, "unit": "Gop/s", "cores": threads,
            "kind": "oracle", "rows_equal_to_gpu": match,
            "sample": f"{rows} full rows of the 4096 x 4096 x 4096 product mod 8388593 "
                      f"({rows * N * K:.3g} multiply-adds, {dt:.1f} s), scaled to Gop/s"}


def i8_source_sha256():
    h = hashlib.sha256()
    for f in I8_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the INT8 S=4 kernel from the committed
    rocprofv3 counter summary, if the kernel source is unchanged since."""
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        sha = i8_source_sha256()
        if kv.get("source_sha256") != sha:
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def freivalds_check(A, B, C0, Cout, alpha, beta, p, trials, seed):
    """Cout == alpha*A*B + beta*C0 (mod p)?  Freivalds' test with `trials`
    random vectors (false acceptance <= p^-trials), in exact uint64 numpy
    arithmetic: every product below is < 2^58."""
    rng = np.random.default_rng(seed)
    A64, B64 = A.astype(np.uint64), B.astype(np.uint64)
    C064, Co64 = C0.astype(np.uint64), Cout.astype(np.uint64)
    P64 = np.uint64(p)
    for _ in range(trials):
        x = rng.integers(0, p, B.shape[1], dtype=np.uint64)
        bx = (B64 @ x) % P64
        abx = (A64 @ bx) % P64
        want = (np.uint64(alpha) * abx % P64 + np.uint64(beta) * ((C064 @ x) % P64) % P64) % P64
        if not np.array_equal((Co64 @ x) % P64, want):
            return False
    return True


def repeated_coeffs(calls, alpha, beta, p):
    """After `calls` applications of C <- alpha*A*B + beta*C to C0:
    C = alpha*(1 + beta + ... + beta^(calls-1))*A*B + beta^calls*C0 (mod p)."""
    geo, bpow = 0, 1
    for _ in range(calls):
        geo = (geo + bpow) % p
        bpow = bpow * beta % p
    return alpha * geo % p, bpow


def headline(torch, ff, args):
    dA, A = residues_dev(torch, (M, K), P, 0x5EED0000 + 2000 + 1)
    dB, B = residues_dev(torch, (K, N), P, 0x5EED0000 + 2000 + 2)
    dC, C = residues_dev(torch, (M, N), P, 0x5EED0000 + 2000 + 3)
    ops = 2.0 * M * N * K
    res = {}
    calls = [0]   # every call below applies C <- 3AB + 5C to the same dC
    for name, opts in (("int8_d7", ff.make_opts(path=ff.FF_PATH_INT8, digit_bits=7,
                                                 winograd_levels=0)),
                       ("int8_d8", ff.make_opts(path=ff.FF_PATH_INT8, digit_bits=8,
                                                 winograd_levels=0)),
                       ("fp64", ff.make_opts(path=ff.FF_PATH_FP64, winograd_levels=0)),
                       ("int8_d7_pairing", ff.make_opts(path=ff.FF_PATH_INT8, digit_bits=7,
                                                         winograd_levels=0, digit_pairing=1))):
        info = ff.ff_plan_query(P, 0, 0, M, N, K, opts)

        def step(opts=opts):
            ff.fgemm(P, dA, dB, dC, ALPHA, BETA, opts=opts)
            calls[0] += 1
        ms, per, prof = time_calls(torch, step, args.steps, args.warmup, ff)
        gemm_ms = prof["gemm_ms"] / max(prof["gemm_launches"], 1)
        slice_ms = prof["slice_ms"] / max(prof["slice_launches"], 1)
        r = {"ms_per_step": ms, "gops": gops(ops, ms), **summarize(per),
             "gemm_kernel_ms": gemm_ms, "slice_kernel_ms": slice_ms,
             "slices": info.slices, "digit_bits": info.digit_bits, "kblock": info.kblock,
             "tile_config": info.tile_config, "digit_products": info.digit_products}
        if info.path == ff.FF_PATH_INT8:
            r["mfma_tops"] = info.digit_products * ops / gemm_ms / 1e9
            r["frac_int8_peak"] = r["mfma_tops"] / PEAK_INT8_TOPS
        else:
            r["mfma_tflops"] = ops / gemm_ms / 1e9
            r["frac_fp64_peak"] = r["mfma_tflops"] / PEAK_FP64_TFLOPS
        r["effective_frac_fp64_peak"] = ops / ms / 1e9 / PEAK_FP64_TFLOPS
        res[name] = r
        log(f"4096 {name}: {ms:.3f} ms/step, {r['gops']:.0f} Gop/s")
    # the same product with one Winograd level (seven half-size digit
    # products, Section 3.2), beside the plain path: effective 2mnk/t
    o = ff.make_opts(path=ff.FF_PATH_INT8, digit_bits=7, winograd_levels=1)

    def wstep():
        ff.fgemm(P, dA, dB, dC, ALPHA, BETA, opts=o)
        calls[0] += 1
    ms, per, _ = time_calls(torch, wstep, args.steps, args.warmup)
    res["int8_d7_winograd1"] = {"ms_per_step": ms, "gops_effective": gops(ops, ms),
                                **summarize(per)}
    log(f"4096 int8_d7_winograd1: {ms:.3f} ms/step, {gops(ops, ms):.0f} Gop/s (2mnk/t)")
    # The timed output itself: after `calls` applications on the same C, by
    # Freivalds against the closed form of the repeated update.
    torch.cuda.synchronize()
    out = dC.cpu().numpy().view(np.uint32)
    a_T, b_T = repeated_coeffs(calls[0], ALPHA, BETA, P)
    ok = freivalds_check(A, B, C, out, a_T, b_T, P, 2, 77)
    res["check"] = {"kind": "freivalds", "trials": 2, "calls_applied": calls[0], "ok": bool(ok)}
    log(f"4096 timed output after {calls[0]} calls: Freivalds {'ok' if ok else 'FAILED'}")
    # one call from C0 on the headline path: rows the CPU leg compares with
    # the oracle
    dC.copy_(torch.from_numpy(C.view(np.int32)).cuda())
    ff.fgemm(P, dA, dB, dC, ALPHA, BETA,
             opts=ff.make_opts(path=ff.FF_PATH_INT8, digit_bits=7, winograd_levels=0))
    torch.cuda.synchronize()
    one_call = dC.cpu().numpy().view(np.uint32).copy()
    return res, (A, B, C, one_call)


def large_modulus(torch, ff, args):
    """4096^3 at p = 2^31 - 1: 8-bit digits (4 slices, 16 products), 7-bit
    digits (5 slices, 25 products) and 7-bit digits with pairing (5 slices,
    15 products of digits and digit sums)."""
    p, n = 2147483647, 4096
    ops = 2.0 * n ** 3
    dA, _ = residues_dev(torch, (n, n), p, 0x5EED0000 + 2500 + 1)
    dB, _ = residues_dev(torch, (n, n), p, 0x5EED0000 + 2500 + 2)
    dC = torch.zeros((n, n), dtype=torch.int32, device="cuda")
    out = {}
    for name, opts in (("int8_d8", ff.make_opts(path=ff.FF_PATH_INT8, digit_bits=8,
                                                 winograd_levels=0)),
                       ("int8_d7", ff.make_opts(path=ff.FF_PATH_INT8, digit_bits=7,
                                                 winograd_levels=0)),
                       ("int8_d7_pairing", ff.make_opts(path=ff.FF_PATH_INT8, digit_bits=7,
                                                         winograd_levels=0, digit_pairing=1))):
        info = ff.ff_plan_query(p, 0, 0, n, n, n, opts)
        ms, per, prof = time_calls(torch, lambda: ff.fgemm(p, dA, dB, dC, 1, 0, opts=opts),
                                   5, 1, ff)
        g = prof["gemm_ms"] / max(1, prof["gemm_launches"])
        out[name] = {"ms": ms, "gops": gops(ops, ms), "gemm_kernel_ms": g,
                     "slices": info.slices, "digit_products": info.digit_products,
                     "frac_int8_peak": info.digit_products * ops / g / 1e9 / PEAK_INT8_TOPS}
        log(f"4096 p=2^31-1 {name}: {ms:.3f} ms ({info.digit_products} digit products)")
    return out


def small_latency(torch, ff, args):
    # m = n = k = 256, p = 65521, alpha = 1, beta = 0
    p, n = 65521, 256
    dA, _ = residues_dev(torch, (n, n), p, 0x5EED0000 + 1000 + 1)
    dB, _ = residues_dev(torch, (n, n), p, 0x5EED0000 + 1000 + 2)
    dC = torch.zeros((n, n), dtype=torch.int32, device="cuda")
    out = {}
    for name, opts in (("fp64", ff.make_opts(path=ff.FF_PATH_FP64, winograd_levels=0)),
                       ("int8", ff.make_opts(path=ff.FF_PATH_INT8, winograd_levels=0))):
        ms, per, _ = time_calls(torch, lambda: ff.fgemm(p, dA, dB, dC, 1, 0, opts=opts),
                                max(50, args.steps), args.warmup)
        out[name] = {"gops": gops(2.0 * n ** 3, ms), **summarize(per)}
        # the same calls made straight on the C entry point with arguments
        # marshalled once: the library's latency without the Python
        # binding's per-call argument handling
        lib = ff.load()
        cargs = (p, 0, 0, n, n, n, 1, dA.data_ptr(), n, dB.data_ptr(), n, 0, dC.data_ptr(), n,
                 ctypes.byref(opts))
        if lib.ff_fgemm_ex(*cargs) != ff.FF_OK:
            raise RuntimeError(lib.ff_last_error().decode())
        ms, per, _ = time_calls(torch, lambda: lib.ff_fgemm_ex(*cargs), max(50, args.steps),
                                args.warmup)
        out[name]["c_entry_point"] = summarize(per)
        log(f"256 {name}: p50 {out[name]['p50_ms'] * 1e3:.1f} us through the binding, "
            f"{out[name]['c_entry_point']['p50_ms'] * 1e3:.1f} us on the C entry point")
    return out


def large_8192(torch, ff, args):
    n = 8192
    ops = 2.0 * n ** 3
    out = {}
    dA, _ = residues_dev(torch, (n, n), 251, 0x5EED0000 + 3000 + 1)
    dB, _ = residues_dev(torch, (n, n), 251, 0x5EED0000 + 3000 + 2)
    dC = torch.zeros((n, n), dtype=torch.int32, device="cuda")
    o = ff.make_opts(path=ff.FF_PATH_INT8, winograd_levels=0)
    ms, per, prof = time_calls(torch, lambda: ff.fgemm(251, dA, dB, dC, 1, 0, opts=o),
                               5, 1, ff)
    g = prof["gemm_ms"] / max(1, prof["gemm_launches"])
    out["p251_int8_direct"] = {"ms": ms, "gops": gops(ops, ms), "gemm_kernel_ms": g,
                               "frac_int8_peak": ops / g / 1e9 / PEAK_INT8_TOPS}
    del dA, dB
    dA, _ = residues_dev(torch, (n, n), P, 0x5EED0000 + 3000 + 3)
    dB, _ = residues_dev(torch, (n, n), P, 0x5EED0000 + 3000 + 4)
    for name, opts in (("p8388593_int8_d7_l0", ff.make_opts(path=ff.FF_PATH_INT8,
                                                             digit_bits=7, winograd_levels=0)),
                       ("p8388593_int8_d7_l1", ff.make_opts(path=ff.FF_PATH_INT8,
                                                             digit_bits=7, winograd_levels=1)),
                       ("p8388593_int8_d7_l2", ff.make_opts(path=ff.FF_PATH_INT8,
                                                             digit_bits=7, winograd_levels=2)),
                       ("p8388593_int8_d8_l0", ff.make_opts(path=ff.FF_PATH_INT8,
                                                             digit_bits=8, winograd_levels=0)),
                       ("p8388593_int8_d8_l1", ff.make_opts(path=ff.FF_PATH_INT8,
                                                             digit_bits=8, winograd_levels=1,
                                                             preadd_mode=2)),
                       ("p8388593_fp64_l0", ff.make_opts(path=ff.FF_PATH_FP64,
                                                          winograd_levels=0)),
                       ("p8388593_fp64_l1", ff.make_opts(path=ff.FF_PATH_FP64,
                                                          winograd_levels=1)),
                       ("p8388593_fp64_l2", ff.make_opts(path=ff.FF_PATH_FP64,
                                                          winograd_levels=2))):
        info = ff.ff_plan_query(P, 0, 0, n, n, n, opts)
        ms, per, _ = time_calls(torch, lambda: ff.fgemm(P, dA, dB, dC, 1, 0, opts=opts), 3, 1)
        out[name] = {"ms": ms, "gops_2mnk": gops(ops, ms), "levels": info.winograd_levels,
                     "slices": info.slices, "preadds_reduced": info.preadds_reduced,
                     "kblock": info.kblock}
        log(f"8192 {name}: {ms:.2f} ms")
    return out


def multimodular(torch, ff, args):
    from paper_cs_0601133_amd import synth
    nmax = 2048
    A = synth.signed_ints(0x5EED0000 + 4000 + 1, (nmax, nmax), 1 << 30)
    B = synth.signed_ints(0x5EED0000 + 4000 + 2, (nmax, nmax), 1 << 30)
    primes = synth.primes_below(1 << 20, 64)
    sizes = [512, 1024, 1536, 2048]
    order = np.random.default_rng(42).permutation(64)
    keep, jobs_i8 = [], []
    total_ops = 0.0
    for idx, pi in enumerate(order):
        p, n = primes[pi], sizes[idx % 4]
        dA = torch.from_numpy(np.mod(A[:n, :n], p).astype(np.uint32).view(np.int32)).cuda()
        dB = torch.from_numpy(np.mod(B[:n, :n], p).astype(np.uint32).view(np.int32)).cuda()
        dC = torch.zeros((n, n), dtype=torch.int32, device="cuda")
        keep.append((dA, dB, dC, p))
        jobs_i8.append(ff.job(p, dA, dB, dC))
        total_ops += 2.0 * n ** 3
    out = {"jobs": 64, "sum_2n3": total_ops}
    stream = torch.cuda.current_stream().cuda_stream
    for name, path in (("int8", ff.FF_PATH_INT8), ("fp64", ff.FF_PATH_FP64)):
        o = ff.make_opts(path=path, stream=stream)
        ms, per, _ = time_calls(torch, lambda: ff.ff_fgemm_batched(jobs_i8, o), 5, 1)
        out[f"{name}_batched"] = {"ms": ms, "gops": gops(total_ops, ms)}
        # the same jobs as separate launches
        solo = ff.make_opts(path=path, winograd_levels=0, stream=stream)

        def one_by_one():
            for j in jobs_i8:
                ff.ff_fgemm_ex(j.p, 0, 0, j.m, j.n, j.k, j.alpha, j.A, j.lda, j.B, j.ldb,
                               j.beta, j.C, j.ldc, solo)
        ms2, _, _ = time_calls(torch, one_by_one, 3, 1)
        out[f"{name}_solo_sum"] = {"ms": ms2, "gops": gops(total_ops, ms2)}
        g = ff.ff_batch_graph_create(jobs_i8, ff.make_opts(path=path))
        ms3, _, _ = time_calls(torch, lambda: ff.ff_batch_graph_launch(g, stream), 5, 1)
        ff.ff_batch_graph_destroy(g)
        out[f"{name}_graph"] = {"ms": ms3, "gops": gops(total_ops, ms3)}
        log(f"batch {name}: batched {ms:.2f} ms, solo {ms2:.2f} ms, graph {ms3:.2f} ms")
    return out


def triangular_solve(torch, ff, args):
    """ftrsm: op(T) X = 3 B mod p, T lower triangular m x m with an invertible
    diagonal, B m x n, solved in place on the path the planner picks for
    the updates (a repeated solve on its own output costs the same).
    Throughput is m^2 n / t: m(m - 1)n/2 multiply-adds, each counted as a
    multiplication and an addition, like 2mnk for a product."""
    from paper_cs_0601133_amd import synth
    out = {}
    for m, n, p in ((4096, 4096, 8388593), (4096, 4096, 65521), (4096, 4096, 2147483647),
                    (8192, 8192, 8388593)):
        T = synth.residues(0x5EED0000 + 7000 + m, (m, m), p)
        d = np.arange(m)
        T[d, d] = 1 + T[d, d] % (p - 1)
        B = synth.residues(0x5EED0000 + 7001 + m, (m, n), p)
        dT = torch.from_numpy(T.view(np.int32)).cuda()
        dB = torch.from_numpy(B.view(np.int32)).cuda()
        del T, B
        ms, per, _ = time_calls(torch, lambda: ff.ftrsm(p, dT, dB, 3, lower=True), 5, 2)
        med = float(np.median(per))
        out[f"m{m}_n{n}_p{p}"] = {"ms": ms, "ms_median_events": med,
                                   "gops_m2n": m * m * n / ms / 1e6}
        log(f"ftrsm m={m} n={n} p={p}: {ms:.3f} ms")
        del dT, dB
    return out


def symmetric_product(torch, ff, args):
    """C <- A diag(D) A^T mod p (Section 6) for m = k = 4096 and 8192,
    p = 8388593, seeded A and D (and without D), next to fgemm computing
    the same product in full (A' A^T with A' = A diag(D) precomputed).
    Throughput is reported as 2 m^2 k / t (what the full product does); the
    symmetric product's classical count is half of it (Section 6)."""
    from paper_cs_0601133_amd import synth
    p = P
    out = {}
    for m in (4096, 8192):
        k = m
        A = synth.residues(0x5EED0000 + 9000 + m, (m, k), p)
        d = synth.residues(0x5EED0000 + 9001 + m, (k,), p)
        AD = (A.astype(np.uint64) * d.astype(np.uint64)[None, :] % p).astype(np.uint32)
        dA = torch.from_numpy(A.view(np.int32)).cuda()
        dD = torch.from_numpy(d.view(np.int32)).cuda()
        dAD = torch.from_numpy(AD.view(np.int32)).cuda()
        dC = torch.zeros((m, m), dtype=torch.int32, device="cuda")
        del A, AD
        ms, _, _ = time_calls(torch, lambda: ff.aat(p, dA, dC, dD), 10, 2)
        ms_nod, _, _ = time_calls(torch, lambda: ff.aat(p, dA, dC), 10, 2)
        ms_full, _, _ = time_calls(torch, lambda: ff.fgemm(p, dA, dAD, dC, transB=True), 10, 2)
        out[f"m{m}_k{k}"] = {"p": p, "ms": ms, "ms_without_D": ms_nod, "ms_fgemm_full": ms_full,
                             "speedup_vs_fgemm": ms_full / ms,
                             "gops_2m2k": 2.0 * m * m * k / ms / 1e6}
        log(f"aat m=k={m}: {ms:.3f} ms ({ms_nod:.3f} without D; full fgemm {ms_full:.3f} ms)")
        del dA, dD, dAD, dC
    return out


def factorisation(torch, ff, args):
    """LQUP (Section 5.1) of a seeded dense n x n matrix of residues, in
    place; each step restores A from a device copy first (a 4 n^2-byte copy,
    under 0.2% of the step).  Throughput is (2/3) n^3 / t, the operation
    count of the factorisation with classical products (Section 5)."""
    from paper_cs_0601133_amd import synth
    out = {}
    for n, p in ((4096, 8388593), (4096, 65521), (8192, 8388593)):
        A = synth.residues(0x5EED0000 + 8000 + n, (n, n), p)
        dA0 = torch.from_numpy(A.view(np.int32)).cuda()
        dA = torch.empty_like(dA0)
        del A
        ranks = []

        def step():
            dA.copy_(dA0)
            ranks.append(ff.lqup(p, dA)[0])
        ms, _, _ = time_calls(torch, step, 3, 1)
        out[f"n{n}_p{p}"] = {"ms": ms, "rank": ranks[-1],
                             "gops_2n3_3": 2.0 * n ** 3 / 3.0 / ms / 1e6}
        log(f"lqup n={n} p={p}: {ms:.2f} ms, rank {ranks[-1]}")
        if n == 4096 and p == 8388593:
            # inverse on the factorisation (Section 6): LQUP, two n x n
            # triangular solves on the identity, a row permutation; the
            # operation count of LQUP plus the solves is 2 n^3
            dX = torch.empty_like(dA0)
            oks = []

            def inv_step():
                dA.copy_(dA0)
                oks.append(ff.inv(p, dA, dX))
            ms_i, _, _ = time_calls(torch, inv_step, 3, 1)
            out[f"inv_n{n}_p{p}"] = {"ms": ms_i, "invertible": bool(oks[-1]),
                                     "gops_2n3": 2.0 * n ** 3 / ms_i / 1e6}
            log(f"inverse n={n} p={p}: {ms_i:.2f} ms")
            del dX
        del dA, dA0
    return out


def serving(torch, ff, args):
    nreq = args.serve_requests
    rng = np.random.default_rng(5)
    primes = [251, 65521, 8388593]
    reqs = []
    for r in range(nreq):
        m, n, k = (int(round(math.exp(rng.uniform(math.log(64), math.log(4096)))))
                   for _ in range(3))
        p = primes[int(rng.integers(0, 3))]
        g = torch.Generator(device="cuda")
        g.manual_seed(0x5EED5000000 + r)
        dA = torch.randint(0, p, (m, k), dtype=torch.int32, device="cuda", generator=g)
        dB = torch.randint(0, p, (k, n), dtype=torch.int32, device="cuda", generator=g)
        dC = torch.randint(0, p, (m, n), dtype=torch.int32, device="cuda", generator=g)
        reqs.append((ff.job(p, dA, dB, dC, 3, 5), (dA, dB, dC, dC.clone(), p), 2.0 * m * n * k))
    torch.cuda.synchronize()
    total_ops = sum(r[2] for r in reqs)
    budget = 24 << 30
    out = {"requests": nreq, "sum_2mnk": total_ops, "hbm_budget_bytes": budget}
    # untimed pass of the same stream first (first launches of the batched
    # kernels, workspace and arena growth), as every other workload settles
    # before it is timed
    srv = ff.ff_server_create(budget)
    ids = [ff.ff_server_submit(srv, r[0]) for r in reqs]
    for i in ids:
        ff.ff_server_wait(srv, i)
    ff.ff_server_destroy(srv)
    # closed loop: everything submitted at once -> capacity
    srv = ff.ff_server_create(budget)
    t0 = time.perf_counter()
    ids = [ff.ff_server_submit(srv, r[0]) for r in reqs]
    for i in ids:
        ff.ff_server_wait(srv, i)
    makespan = time.perf_counter() - t0
    st = ff.ff_server_stats(srv)
    ff.ff_server_destroy(srv)
    cap = nreq / makespan
    out["closed_loop"] = {"makespan_s": makespan, "req_per_s": cap, "gops": total_ops / makespan / 1e9,
                          "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                          "max_inflight": st["max_inflight"]}
    log(f"serve closed loop: {makespan*1e3:.1f} ms, {cap:.0f} req/s")
    for load in (0.5, 0.9):
        rate = load * cap
        arr = np.cumsum(np.random.default_rng(6).exponential(1.0 / rate, nreq))
        srv = ff.ff_server_create(budget)
        t0 = time.perf_counter()
        ids = []
        for r, t in zip(reqs, arr):
            while time.perf_counter() - t0 < t:
                pass
            ids.append(ff.ff_server_submit(srv, r[0]))
        for i in ids:
            ff.ff_server_wait(srv, i)
        dt = time.perf_counter() - t0
        st = ff.ff_server_stats(srv)
        ff.ff_server_destroy(srv)
        out[f"poisson_{load}"] = {"offered_req_per_s": rate, "gops": total_ops / dt / 1e9,
                                  "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                                  "max_inflight": st["max_inflight"]}
        log(f"serve poisson {load}: p50 {st['p50_ms']:.2f} ms p99 {st['p99_ms']:.2f} ms")
    # every request's result after the four runs (C <- 3AB + 5C applied
    # four times: the untimed pass, the closed loop and two Poisson
    # streams), by Freivalds against its initial C
    torch.cuda.synchronize()
    good = 0
    for i, (_, (dA, dB, dC, dC0, p), _) in enumerate(reqs):
        a_T, b_T = repeated_coeffs(4, 3, 5, p)
        host = [t.cpu().numpy().view(np.uint32) for t in (dA, dB, dC0, dC)]
        good += freivalds_check(host[0], host[1], host[2], host[3], a_T, b_T, p, 1, 1000 + i)
    out["check"] = {"kind": "freivalds", "trials": 1, "requests": nreq, "ok": int(good)}
    log(f"serve: {good} of {nreq} results pass Freivalds")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_cs_0601133_amd import ffgemm as ff

    torch.cuda.set_device(0)
    ff.ff_init()
    if args.ftrsm_only:
        print(json.dumps({"workloads": {"ftrsm": triangular_solve(torch, ff, args)}}))
        return
    if args.aat_only:
        print(json.dumps({"workloads": {"aat": symmetric_product(torch, ff, args)}}))
        return
    if args.lqup_only:
        print(json.dumps({"workloads": {"lqup": factorisation(torch, ff, args)}}))
        return
    if args.n8192_only:
        print(json.dumps({"workloads": {"n8192": large_8192(torch, ff, args)}}))
        return
    if args.latency_only:
        print(json.dumps({"workloads": {"n256_p65521_latency": small_latency(torch, ff, args)}}))
        return
    if args.multimodular_only:
        print(json.dumps({"workloads": {"multimodular_64_jobs": multimodular(torch, ff, args)}}))
        return
    if args.serving_only:
        print(json.dumps({"workloads": {"serving": serving(torch, ff, args)}}))
        return
    global SETTLE_S
    SETTLE_S = args.settle_s
    paths, (A, B, C, one_call) = headline(torch, ff, args)
    check = paths.pop("check")
    head = paths["int8_d7"]
    ops = 2.0 * M * N * K
    line = {
        "metric": "modular GEMM Gop/s (2mnk/t, bit-exact) INT8-sliced vs FP64; p50/p99 latency",
        "value": head["gops"],
        "unit": "Gop/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_s": args.settle_s,
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
                     "frac": head["frac_int8_peak"], "traffic": measured_traffic(),
                     "kernel": "k_fgemm_i8 (S=4)", "ops_per_launch": 16 * ops},
        "paths": paths,
        "check": check,
        "int8_vs_fp64_speedup": paths["fp64"]["ms_per_step"] / head["ms_per_step"],
    }
    if args.headline_only:
        # plain copy of a known size: the reference that scales the HBM
        # counters of a profiler run
        src = torch.ones(64 << 20, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_probe_bytes"] = src.numel() * 4
    if not args.headline_only:
        line["workloads"] = {
            "n256_p65521_latency": small_latency(torch, ff, args),
            "n4096_p2147483647": large_modulus(torch, ff, args),
            "n8192": large_8192(torch, ff, args),
            "multimodular_64_jobs": multimodular(torch, ff, args),
            "ftrsm": triangular_solve(torch, ff, args),
            "lqup": factorisation(torch, ff, args),
            "aat": symmetric_product(torch, ff, args),
            "serving": serving(torch, ff, args),
        }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(A, B, C, args.cpu_seconds, one_call)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
