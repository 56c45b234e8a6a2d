"""Benchmark of the checksum-protected FP64 GEMM on one MI355X.

One step = one protected GEMM call C := alpha A B + beta C (fused encode,
maintained checksums, reference sums, verify, locate/correct) on the square
FP64 workload n = m = k = 8192, alpha = 1.5, beta = 0.5, A/B/C i.i.d.
U[-1,1], with seeded bit flips at one per 2^32 multiply-adds (128 faults, at
most one per tile).  Inputs are resident in HBM before timing starts.

Printed (one JSON line): TFLOP/s of the protected call with faults injected,
the same kernel with ABFT compiled out, the overhead %, a roofline object for
the GEMM kernel (FP64 MFMA bound) and the CPU oracle's throughput on a bounded
sample of the same workload.  Extra sizes of the FP64 sweep and the rank-k
shapes are reported with --sweep.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_F64_MFMA = 78.6  # TFLOP/s, MI355X dense FP64 matrix
# HBM bytes per launch of the protected product kernel (tile configuration 5,
# encode pass) at n = 8192 from rocprofv3 FETCH_SIZE / WRITE_SIZE runs, scaled
# by a plain-copy calibration (profiles/dgemm_abft_n8192_traffic.md); it must be
# re-measured whenever that kernel changes
TRAFFIC_F64_N8192 = 1.729e10


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--n", type=int, default=8192)
    p.add_argument("--tile", type=int, default=0)
    p.add_argument("--sweep", action="store_true", help="also time the FP64 size sweep and rank-k shapes")
    p.add_argument("--tiles", action="store_true", help="time every FP64 tile configuration at --n")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-configs", action="store_true", help="skip the other workloads (cfg 1, 3, 4, 5)")
    return p.parse_args()


def device_operands(torch, ftgemm, m, n, k, seed, ta=0, tb=0):
    """U[-1,1] operands drawn on the host (numpy PCG64) and copied to HBM."""
    from paper_2104_00897_amd import inputs
    A, B, C = inputs.gemm_operands_f64(m, n, k, seed=seed, ta=ta, tb=tb)
    return ftgemm.to_device(A), ftgemm.to_device(B), ftgemm.to_device(C), (A, B, C)


def time_calls(torch, fn, steps, warmup, kernel_timer=None):
    """ms per call over `steps` calls (HIP events on the current stream).  With a
    handle as kernel_timer, the library also times its product kernel launches
    (events on the same stream) and the list kernel_timer_out gets their mean."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if kernel_timer is not None:
        kernel_timer.timing(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    if kernel_timer is not None:
        n, t = kernel_timer.timing_read()
        kernel_timer.timing(False)
        KERNEL_MS.append(t / max(1, n))
    return e0.elapsed_time(e1) / steps  # ms per call


KERNEL_MS: list = []  # mean product-kernel duration of each timed run with a kernel timer


def measure(torch, ftgemm, h, m, n, k, alpha, beta, ta, tb, steps, warmup, tile, seed=0):
    dA, dB, dC, host = device_operands(torch, ftgemm, m, n, k, seed, ta, tb)
    rate = 2.0 ** -32
    faults = math.ceil(m * n * k * rate)
    cfg_p = ftgemm.make_config(tile=tile, seed=1234, per_mac_rate=rate)
    cfg_u = ftgemm.make_config(abft=False, tile=tile)
    cfg_0 = ftgemm.make_config(tile=tile)

    def call(cfg):
        return lambda: ftgemm.gemm_f64(h, dA, dB, dC, alpha, beta, ta, tb, cfg=cfg)

    # alternate protected / unprotected to cancel clock drift
    tp, tu, t0 = [], [], []
    h.reset()
    KERNEL_MS.clear()
    for _ in range(2):
        tp.append(time_calls(torch, call(cfg_p), steps, warmup, kernel_timer=h))
        tu.append(time_calls(torch, call(cfg_u), steps, warmup))
        t0.append(time_calls(torch, call(cfg_0), steps, warmup))
    kernel_ms = float(np.median(KERNEL_MS))
    rep = h.read()
    flops = 2.0 * m * n * k
    ms_p, ms_u, ms_0 = float(np.median(tp)), float(np.median(tu)), float(np.median(t0))
    return {
        "m": m, "n": n, "k": k, "ta": ta, "tb": tb,
        "tile": tile or h.tune_get(ftgemm.F64, m, n, k),
        "ms_protected": ms_p, "ms_unprotected": ms_u, "ms_protected_no_faults": ms_0,
        "tflops_protected": flops / ms_p / 1e9,
        "tflops_unprotected": flops / ms_u / 1e9,
        "tflops_protected_no_faults": flops / ms_0 / 1e9,
        "overhead_pct": 100.0 * (ms_p / ms_u - 1.0),
        "overhead_no_faults_pct": 100.0 * (ms_0 / ms_u - 1.0),
        "kernel_ms_protected": kernel_ms,
        "faults_per_call": faults,
        "injected": rep.injected, "corrected": rep.corrected_subtract + rep.corrected_recompute,
        "uncorrectable": rep.uncorrectable, "detected": rep.detected,
    }, host


def timed_ab(torch, fns, steps, warmup, rounds=2):
    """Median ms per call of each function, alternating them round by round."""
    out = {name: [] for name in fns}
    for _ in range(rounds):
        for name, fn in fns.items():
            out[name].append(time_calls(torch, fn, steps, warmup))
    return {name: float(np.median(v)) for name, v in out.items()}


def cfg1_latency(torch, ftgemm, h, steps):
    """256^3 FP64, alpha = 1, beta = 0, U[-1,1] seed 0, 4 flips in distinct slots
    (the library's default tile for this shape, 64 x 64: 16 slots): microseconds
    per protected call (launch-latency bound)."""
    from paper_2104_00897_amd import inputs
    A, B, _ = inputs.gemm_operands_f64(256, 256, 256, seed=0, with_c=False)
    dA, dB = ftgemm.to_device(A), ftgemm.to_device(B)
    dC = torch.zeros((256, 256), dtype=torch.float64, device="cuda")
    cp = ftgemm.make_config(seed=0, n_faults=4)
    cu = ftgemm.make_config(abft=False)
    t = timed_ab(torch, {"p": lambda: ftgemm.gemm_f64(h, dA, dB, dC, 1.0, 0.0, cfg=cp),
                         "u": lambda: ftgemm.gemm_f64(h, dA, dB, dC, 1.0, 0.0, cfg=cu)}, steps * 10, 5)
    return {"workload": "FP64 256^3 NN, 4 flips", "tile": h.tune_get(ftgemm.F64, 256, 256, 256),
            "us_protected": 1e3 * t["p"], "us_unprotected": 1e3 * t["u"]}


def lowp_operands(torch, kind, rows, cols, seed, std=1.0):
    """Column-major (rows x cols) operand as a (cols x rows) device tensor: N(0, std^2)
    rounded to bf16, or absmax-scaled e4m3fn codes with their per-tensor scale."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    x = torch.randn((cols, rows), generator=g, device="cuda", dtype=torch.float32) * std
    if kind == "bf16":
        return x.to(torch.bfloat16).view(torch.int16), None
    s = x.abs().max() / 448.0
    try:
        q = (x / s).to(torch.float8_e4m3fn).view(torch.uint8)
    except (RuntimeError, TypeError):
        from paper_2104_00897_amd import inputs
        q = torch.from_numpy(inputs.to_e4m3_bits((x / s).double().cpu().numpy())).cuda()
    return q, s.reshape(1).float()


def cfg3_lowp(torch, ftgemm, h, kind, steps, n=8192):
    """8192^3 NN, alpha = 1, beta = 0, N(0,1) operands (bf16, or e4m3fn with absmax
    scales), 16 flips of FP32 accumulator bits 13..30 per call."""
    dA, sa = lowp_operands(torch, kind, n, n, 1)
    dB, sb = lowp_operands(torch, kind, n, n, 2)
    dC = torch.empty((n, n), dtype=torch.float32, device="cuda")
    ab = ftgemm.BF16 if kind == "bf16" else ftgemm.F8_E4M3
    cfgs = {"p": ftgemm.make_config(seed=7, n_faults=16, bit_lo=13, bit_hi=30),
            "u": ftgemm.make_config(abft=False), "p0": ftgemm.make_config()}
    fns = {k: (lambda c=c: ftgemm.gemm_lowp(h, dA, dB, dC, 1.0, 0.0, 0, 0, ab, sa, sb, c))
           for k, c in cfgs.items()}
    h.reset()
    t = timed_ab(torch, fns, steps, 2)
    rep = h.read()
    fl = 2.0 * n ** 3
    peak = 2500.0 if kind == "bf16" else 5000.0
    return {"workload": f"{kind} {n}^3 NN -> FP32, 16 flips/call", "ms_protected": t["p"],
            "ms_unprotected": t["u"], "ms_protected_no_faults": t["p0"],
            "tflops_protected": fl / t["p"] / 1e9, "tflops_unprotected": fl / t["u"] / 1e9,
            "overhead_pct": 100.0 * (t["p"] / t["u"] - 1.0), "frac_of_peak_protected": fl / t["p"] / 1e9 / peak,
            "faults": {"injected": rep.injected, "corrected": rep.corrected_subtract + rep.corrected_recompute,
                       "detected": rep.detected, "uncorrectable": rep.uncorrectable}}


def cfg4_ftlinear(torch, ftgemm, h, steps):
    """One training step of FTLinear (bf16): tokens 8192, in 4096, out 4096; forward,
    input and weight gradients; 16 flips (bits 24..30) in each backward GEMM."""
    from paper_2104_00897_amd import ftlinear
    T, din, dout = 8192, 4096, 4096
    g = torch.Generator(device="cuda").manual_seed(0)
    X = (torch.randn((T, din), generator=g, device="cuda") * 0.02).to(torch.bfloat16).requires_grad_(True)
    W = (torch.randn((dout, din), generator=g, device="cuda") * 0.02).to(torch.bfloat16).requires_grad_(True)
    G = torch.randn((T, dout), generator=g, device="cuda").to(torch.bfloat16)
    cb = ftgemm.make_config(seed=4, n_faults=16, bit_lo=24, bit_hi=30)
    cu = ftgemm.make_config(abft=False)

    def step(cf, cbw):
        X.grad = None
        W.grad = None
        ftlinear.ft_linear(X, W, h, cf, cbw).backward(G)

    h.reset()
    t = timed_ab(torch, {"p": lambda: step(None, cb), "u": lambda: step(cu, cu)}, steps, 2)
    rep = h.read()
    fl = 3 * 2.0 * T * din * dout
    return {"workload": "FTLinear bf16 step, tokens 8192, 4096 -> 4096, 16 flips per backward GEMM",
            "ms_protected": t["p"], "ms_unprotected": t["u"], "tflops_protected": fl / t["p"] / 1e9,
            "tflops_unprotected": fl / t["u"] / 1e9, "overhead_pct": 100.0 * (t["p"] / t["u"] - 1.0),
            "faults": {"injected": rep.injected, "corrected": rep.corrected_subtract + rep.corrected_recompute,
                       "uncorrectable": rep.uncorrectable}}


def cfg5_batched(torch, ftgemm, h, steps):
    """512 FP64 problems, m, n, k log-uniform in [32, 2048] (seed 7), alpha = 1,
    beta = 0, U[-1,1] operands, 0-2 flips per problem (U{0,1,2}, seed 7), one
    persistent launch; eager and hipGraph-replayed."""
    from paper_2104_00897_amd import inputs
    sizes = inputs.log_uniform_sizes(512, 32, 2048, 7)
    faults = np.random.default_rng(7).integers(0, 3, size=len(sizes))
    g = torch.Generator(device="cuda").manual_seed(7)
    keep, probs = [], []
    for m, n, k in sizes:
        A = torch.rand((k, m), generator=g, device="cuda", dtype=torch.float64) * 2 - 1
        B = torch.rand((n, k), generator=g, device="cuda", dtype=torch.float64) * 2 - 1
        C = torch.zeros((n, m), device="cuda", dtype=torch.float64)
        keep.append((A, B, C))
        probs.append(ftgemm.batch_problem(A, B, C, 1.0, 0.0))
    plan = ftgemm.BatchPlan(probs)
    cp = ftgemm.make_config(tile=3, seed=7, n_faults=1)
    cu = ftgemm.make_config(abft=False, tile=3)
    stream = ftgemm.current_stream_ptr
    fl = float(sum(2.0 * m * n * k for m, n, k in sizes))
    h.reset()
    t = timed_ab(torch, {"p": lambda: h.dgemm_batched(plan, stream(), cp, faults),
                         "u": lambda: h.dgemm_batched(plan, stream(), cu)}, steps, 2)
    rep = h.read()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        h.dgemm_batched(plan, stream(), cp, faults)
    tg = time_calls(torch, gr.replay, steps, 2)
    torch.cuda.synchronize()
    del gr
    return {"workload": "512 FP64 problems, m,n,k log-uniform [32, 2048], seed 7, 0-2 flips each",
            "gflop": fl / 1e9, "ms_protected": t["p"], "ms_unprotected": t["u"], "ms_protected_graph": tg,
            "tflops_protected": fl / t["p"] / 1e9, "tflops_unprotected": fl / t["u"] / 1e9,
            "overhead_pct": 100.0 * (t["p"] / t["u"] - 1.0),
            "faults": {"injected": rep.injected, "corrected": rep.corrected_subtract + rep.corrected_recompute,
                       "uncorrectable": rep.uncorrectable}}


def cpu_baseline(host, k):
    """The oracle's ABFT procedure (single thread) on a bounded sample: the
    leading 1536 x 1536 block of C with the full k of the workload."""
    import oracle
    A, B, C = host
    ms = ns = 1536
    As = np.asfortranarray(A[:ms, :])
    Bs = np.asfortranarray(B[:, :ns])
    Cs = np.asfortranarray(C[:ms, :ns])
    t0 = time.perf_counter()
    oracle.abft(As, Bs, Cs, 1.5, 0.5, bm=128, bn=128)
    dt = time.perf_counter() - t0
    flops = 2.0 * ms * ns * k
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle.abft on the leading {ms}x{ns} block of C with k={k} "
                      f"(bm=bn=128 tiles, same operands): {flops / 1e9:.2f} GFLOP in {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2104_00897_amd import ftgemm

    h = ftgemm.Handle(capacity=16384)
    n = args.n
    res, host = measure(torch, ftgemm, h, n, n, n, 1.5, 0.5, 0, 0, args.steps, args.warmup, args.tile)
    flops = 2.0 * n ** 3
    achieved = res["tflops_protected"]
    # roofline of the protected product kernel itself: algorithmic flops per
    # launch (2 n^3) over its mean launch duration (library-recorded events)
    kernel_tf = flops / res["kernel_ms_protected"] / 1e9
    line = {
        "metric": "FT-GEMM TFLOP/s & ABFT overhead % vs unprotected, faults injected, 1 GPU",
        "value": round(achieved, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_protected"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"FP64 ABFT DGEMM NN m=n=k={n}, alpha=1.5, beta=0.5, U[-1,1], "
                               f"1 bit flip per 2^32 MACs ({res['faults_per_call']} per call)",
                   "tile": res["tile"]},
        "abft_overhead_pct": round(res["overhead_pct"], 2),
        "abft_overhead_no_faults_pct": round(res["overhead_no_faults_pct"], 2),
        "unprotected_tflops": round(res["tflops_unprotected"], 3),
        "faults": {"injected": res["injected"], "corrected": res["corrected"],
                   "uncorrectable": res["uncorrectable"]},
        "roofline": {"bound": "mfma", "achieved": round(kernel_tf, 3), "peak": PEAK_F64_MFMA,
                     "unit": "TFLOP/s", "frac": round(kernel_tf / PEAK_F64_MFMA, 4),
                     "traffic": TRAFFIC_F64_N8192 if n == 8192 else None,
                     "kernel": "protected FP64 product kernel (128x128 tile, 8 waves)",
                     "kernel_ms": round(res["kernel_ms_protected"], 4)},
    }
    if args.tiles:
        for t in (1, 2, 3, 4, 5):
            r, _ = measure(torch, ftgemm, h, n, n, n, 1.5, 0.5, 0, 0, max(3, args.steps // 2), 1, t)
            print(json.dumps({"tile_sweep": r}), file=sys.stderr, flush=True)
    if args.sweep:
        sweep = []
        for nn in (1024, 2048, 4096, 8192, 16384):
            r, _ = measure(torch, ftgemm, h, nn, nn, nn, 1.5, 0.5, 0, 0, max(3, args.steps // 2), 1, 0)
            sweep.append(r)
            print(json.dumps({"sweep": r}), file=sys.stderr, flush=True)
        for kk in (128, 256, 512):
            for ta in (0, 1):
                r, _ = measure(torch, ftgemm, h, 16384, 16384, kk, 1.5, 0.5, ta, 0, args.steps, 1, 0)
                sweep.append(r)
                print(json.dumps({"sweep": r}), file=sys.stderr, flush=True)
        line["sweep"] = sweep
    if not args.no_configs:
        cf = {}
        for name, fn in [("cfg1", lambda: cfg1_latency(torch, ftgemm, h, args.steps)),
                         ("cfg3_bf16", lambda: cfg3_lowp(torch, ftgemm, h, "bf16", args.steps)),
                         ("cfg3_fp8", lambda: cfg3_lowp(torch, ftgemm, h, "fp8", args.steps)),
                         ("cfg4", lambda: cfg4_ftlinear(torch, ftgemm, h, max(2, args.steps // 2))),
                         ("cfg5", lambda: cfg5_batched(torch, ftgemm, h, args.steps))]:
            cf[name] = fn()
            print(json.dumps({name: cf[name]}), file=sys.stderr, flush=True)
        line["configs"] = cf
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(host, n)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
