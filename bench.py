"""Benchmark of the checksum-protected FP64 GEMM on one MI355X.

One step = one protected GEMM call C := alpha A B + beta C (encode pass,
maintained checksums, reference sums, verify, locate/correct) on the square
FP64 workload n = m = k = 16384 (the largest of the FP64 sweep), alpha = 1.5,
beta = 0.5, A/B/C i.i.d. U[-1,1], with seeded bit flips at one per 2^32
multiply-adds (1024 faults, at most one per tile).  Inputs are resident in
HBM before timing starts.

Printed (one JSON line): TFLOP/s of the protected call with faults injected,
the same kernel with ABFT compiled out, the overhead %, a roofline object for
the protected product kernel (FP64 MFMA bound), the rest of the FP64 sweep
(1024..8192 and the rank-k updates m = n = 16384, k = 128/256/512, NN and
TN), the other workloads (FP64 256^3 latency, BF16/FP8 8192^3 with the
false-positive campaign, the FTLinear step, 512 batched problems) and the CPU
oracle's throughput on a bounded sample of the headline workload.
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
PEAK_HBM = 8000.0     # GB/s
# HBM bytes per launch of the protected product kernel by problem size, from
# rocprofv3 FETCH_SIZE / WRITE_SIZE runs scaled by a plain-copy calibration
# (profiles/dgemm_abft_*_traffic.md); an entry is dropped whenever that kernel
# changes, and the line then reports null until it is measured again
TRAFFIC_F64: dict = {16384: 1.5406e11}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--n", type=int, default=16384)
    p.add_argument("--tile", type=int, default=0)
    p.add_argument("--no-sweep", action="store_true", help="skip the FP64 size sweep and rank-k shapes")
    p.add_argument("--fp-calls", type=int, default=1000,
                   help="fault-free calls of the BF16/FP8 false-positive campaign")
    p.add_argument("--only", default="", help="comma list of legs to run among cfg1,cfg3,cfg4,cfg5,unfused,level3,dmr")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only copy 1 GiB between device buffers three times (reference for HBM counters)")
    p.add_argument("--tiles", action="store_true", help="time every FP64 tile configuration at --n")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-configs", action="store_true", help="skip the other workloads (cfg 1, 3, 4, 5)")
    p.add_argument("--calibrate", type=int, default=0,
                   help="only measure the binary32 threshold noise over this many calls per input family")
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
    bytes_alg = 8.0 * (m * k + k * n + 2 * m * n)  # A, B read, C read and written
    return {
        "m": m, "n": n, "k": k, "ta": ta, "tb": tb,
        "tile": tile or h.tune_get(ftgemm.F64, m, n, k),
        "kernel_frac_of_fp64_peak": flops / kernel_ms / 1e9 / PEAK_F64_MFMA,
        "kernel_hbm_gbs_algorithmic": bytes_alg / kernel_ms / 1e6,
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
    """Median ms per call of each function, alternating them round by round.  The
    order rotates from round to round (at least one round per function), so that
    no function always runs first, right after whatever preceded the leg."""
    out = {name: [] for name in fns}
    names = list(fns)
    for r in range(max(rounds, len(names))):
        for name in names[r % len(names):] + names[:r % len(names)]:
            out[name].append(time_calls(torch, fns[name], steps, warmup))
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


def lowp_operands(torch, kind, rows, cols, seed, std=1.0, dist="normal"):
    """Column-major (rows x cols) operand as a (cols x rows) device tensor: N(0, std^2)
    (or U[0, std) with dist="uniform01") rounded to bf16, or absmax-scaled e4m3fn
    codes with their per-tensor scale."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    if dist == "uniform01":
        x = torch.rand((cols, rows), generator=g, device="cuda", dtype=torch.float32) * std
    else:
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


def lowp_values(torch, q, s, kind):
    """Exact binary64 values (host, rows x cols) of a device operand made by lowp_operands."""
    if kind == "bf16":
        return q.view(torch.bfloat16).double().cpu().numpy().T
    from paper_2104_00897_amd import inputs
    return inputs.e4m3_table()[q.cpu().numpy()].T


def acc32_line_tau(a, b, lam, i, j, bm=128, bn=128):
    """The binary32 paths' threshold at element (i, j) (alpha = 1, beta = 0), the
    larger of its tile row's and column's: 2 lam sqrt(k + len + 8) 2^-24 M (1 + 2^-20)
    with the magnitude bounds the kernels use (sum_p |a_ip|) max_p (sum_{j in J} |b_pj|)
    and (sum_p |b_pj|) max_p (sum_{i in I} |a_ip|); a, b: |op(A)|, |op(B)|."""
    m, k = a.shape
    n = b.shape[1]
    i0, j0 = (i // bm) * bm, (j // bn) * bn
    R, Q = min(bm, m - i0), min(bn, n - j0)
    mr = a[i, :].sum() * b[:, j0:j0 + Q].sum(axis=1).max()
    mc = b[:, j].sum() * a[i0:i0 + R, :].sum(axis=0).max()
    g = lambda nt: 2.0 * lam * math.sqrt(nt) * 2.0 ** -24 * (1 + 2.0 ** -20)
    return max(g(k + Q + 8) * mr, g(k + R + 8) * mc)


def fault_classes(rep, a, b, lam, scale=1.0):
    """Splits the logged injections by the detectability rule: a flip whose error
    clears 4 tau of its element must be corrected (else it is missed); a smaller
    one that stays uncorrected is masked.  a, b: |op(A)|, |op(B)| in the stored
    (code) domain; `scale` carries the FP8 per-tensor scales to the output."""
    fixed = {(r["row"], r["col"]) for r in rep.records if r["kind"] in (1, 2)}
    seen, out = set(), {"distinct": 0, "must_correct": 0, "corrected": 0, "masked": 0, "missed": 0}
    taus = []
    for g in rep.inject_log:
        key = (g["row"], g["col"], g["bit"])
        if key in seen:
            continue
        seen.add(key)
        out["distinct"] += 1
        tau = scale * acc32_line_tau(a, b, lam, g["row"], g["col"])
        taus.append(tau / max(1e-300, abs(g["old_val"]) * scale))
        d = abs(g["new_val"] - g["old_val"]) * scale
        ok = (g["row"], g["col"]) in fixed
        out["corrected"] += ok
        if not math.isfinite(d) or d >= 4.0 * tau:
            out["must_correct"] += 1
            out["missed"] += not ok
        elif not ok:
            out["masked"] += 1
    out["median_tau_over_abs_c"] = float(np.median(taus)) if taus else None
    return out


def cfg3_lowp(torch, ftgemm, h, kind, steps, n=8192, fp_calls=1000):
    """8192^3 NN, alpha = 1, beta = 0, N(0,1) operands (bf16, or e4m3fn with absmax
    scales), 16 flips of FP32 accumulator bits 13..30 per call; then `fp_calls`
    fault-free calls (the false-positive campaign) and the detection floor."""
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
    # the kernels fold the scales into alpha in binary32: alpha s_A s_B
    scale = float(np.float32(np.float32(sa.item()) * np.float32(sb.item()))) if sa is not None else 1.0
    a = np.abs(lowp_values(torch, dA, sa, kind))
    b = np.abs(lowp_values(torch, dB, sb, kind))
    lam = ftgemm.default_lambda()
    classes = fault_classes(rep, a, b, lam, scale)
    # error of the FP32 result against the binary64 product of the same values (the
    # FP64 path, itself held to the oracle at 1e-12): normwise and componentwise
    f0 = fns["p0"]
    f0()
    A64 = (dA.view(torch.bfloat16) if kind == "bf16" else dA.view(torch.float8_e4m3fn)).double()
    B64 = (dB.view(torch.bfloat16) if kind == "bf16" else dB.view(torch.float8_e4m3fn)).double()
    C64 = torch.empty((n, n), dtype=torch.float64, device="cuda")
    M64 = torch.empty((n, n), dtype=torch.float64, device="cuda")
    ftgemm.gemm_f64(h, A64, B64, C64, scale, 0.0)
    ftgemm.gemm_f64(h, A64.abs(), B64.abs(), M64, scale, 0.0)
    torch.cuda.synchronize()
    diff = dC.double() - C64
    err = {"normwise_rel": float(torch.linalg.norm(diff) / torch.linalg.norm(C64)),
           "max_componentwise": float((diff.abs() / M64).max()),
           "bound_componentwise": 2.0 * (n + 2) * 2.0 ** -24}
    del A64, B64, C64, M64, diff
    # false-positive campaign: fault-free calls at the default threshold
    h.reset()
    for _ in range(fp_calls):
        f0()
    torch.cuda.synchronize()
    fp = h.read()
    # verification intervals: the product as rank-K_c updates of C, fault-free
    ivl = {kc: (lambda c=ftgemm.make_config(interval_k=kc): ftgemm.gemm_lowp(h, dA, dB, dC, 1.0, 0.0, 0, 0, ab,
                                                                           sa, sb, c))
           for kc in (4096, 2048, 1024)}
    h.reset()
    ti = timed_ab(torch, ivl, max(2, steps // 2), 1)
    ivl_flags = h.read().detected
    return {"workload": f"{kind} {n}^3 NN -> FP32, 16 flips/call", "ms_protected": t["p"],
            "ms_unprotected": t["u"], "ms_protected_no_faults": t["p0"],
            "tflops_protected": fl / t["p"] / 1e9, "tflops_unprotected": fl / t["u"] / 1e9,
            "overhead_pct": 100.0 * (t["p"] / t["u"] - 1.0), "frac_of_peak_protected": fl / t["p"] / 1e9 / peak,
            "faults": {"injected": rep.injected, "corrected": rep.corrected_subtract + rep.corrected_recompute,
                       "detected": rep.detected, "uncorrectable": rep.uncorrectable,
                       "per_distinct_flip": classes},
            "lambda": lam, "error_vs_fp64": err,
            "false_positives": {"calls": fp_calls, "flagged_slots": fp.detected,
                                "checks_per_call": 2 * n * (n // 128),
                                "max_pass_ratio": fp.max_pass_ratio},
            "intervals": {"ms_protected_no_faults": {str(kc): ms for kc, ms in ti.items()},
                          "flagged_slots": ivl_flags}}


def calibrate_lambda(torch, ftgemm, h, calls):
    """Noise of the binary32 paths against the threshold at lambda = 1: the largest
    |delta| / tau over `calls` fault-free calls per input family.  Since tau is
    linear in lambda, that ratio is the smallest lambda with no false positive in
    the campaign."""
    n = 8192
    out = []
    fams = [("bf16", "normal", 1.0, 1.0), ("fp8", "normal", 1.0, 1.0),
            ("bf16", "uniform01", 1.0, 1.0), ("fp8", "uniform01", 1.0, 1.0),
            ("bf16", "normal", 0.02, 1.0)]
    for kind, dist, sa_std, sb_std in fams:
        dA, sa = lowp_operands(torch, kind, n, n, 11, sa_std, dist)
        dB, sb = lowp_operands(torch, kind, n, n, 12, sb_std, dist)
        dC = torch.empty((n, n), dtype=torch.float32, device="cuda")
        ab = ftgemm.BF16 if kind == "bf16" else ftgemm.F8_E4M3
        cfg = ftgemm.make_config(lam=1.0)
        h.reset()
        for _ in range(calls):
            ftgemm.gemm_lowp(h, dA, dB, dC, 1.0, 0.0, 0, 0, ab, sa, sb, cfg)
        torch.cuda.synchronize()
        rep = h.read()
        row = {"kind": kind, "dist": dist, "std": [sa_std, sb_std], "calls": calls,
               "flagged_at_lambda_1": rep.detected, "max_pass_ratio_at_lambda_1": rep.max_pass_ratio}
        print(json.dumps({"calibrate": row}), file=sys.stderr, flush=True)
        out.append(row)
        del dA, dB, dC
    return out


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


def unfused_comparison(torch, ftgemm, h, steps, sizes=(4096, 8192, 16384), kc_online=512):
    """The fused protected product against the unfused comparator (the online ABFT
    of section 5.1 built around the unprotected product, whole-matrix checksums):
    FP64 NN n^3, alpha = 1.5, beta = 0.5, U[-1,1], one flip per rank-K_c slab in
    both (exponent bits, so each is corrected).  The fused product runs with one
    check per tile and online (per-tile checks every K_c = 512 steps); the
    unfused scheme runs offline (one slab) and online (K_c = 512); its cost is
    compared with the paper's
    model (6 + 2K/K_c) P_mm / (n P_mv), P_mm the unprotected product's rate and
    P_mv = 2 flop per 8 bytes at the 8 TB/s HBM peak."""
    rows = []
    for n in sizes:
        dA, dB, dC, _ = device_operands(torch, ftgemm, n, n, n, seed=n + 3)
        fl = 2.0 * n ** 3
        nint = n // kc_online
        inj = dict(seed=5, bit_lo=52, bit_hi=62)
        fns = {
            "unprotected": lambda: ftgemm.gemm_f64(h, dA, dB, dC, 1.5, 0.5, cfg=ftgemm.make_config(abft=False)),
            "fused": lambda: ftgemm.gemm_f64(h, dA, dB, dC, 1.5, 0.5,
                                             cfg=ftgemm.make_config(n_faults=nint, **inj)),
            # the fused product with the same verification interval (online, per tile)
            "fused_online": lambda: ftgemm.gemm_f64(h, dA, dB, dC, 1.5, 0.5,
                                                    cfg=ftgemm.make_config(interval_k=kc_online, n_faults=nint,
                                                                           **inj)),
            "unfused_offline": lambda: ftgemm.gemm_f64_unfused(h, dA, dB, dC, 1.5, 0.5,
                                                               cfg=ftgemm.make_config(n_faults=1, **inj)),
            "unfused_online": lambda: ftgemm.gemm_f64_unfused(
                h, dA, dB, dC, 1.5, 0.5, cfg=ftgemm.make_config(interval_k=kc_online, n_faults=nint, **inj)),
            "unfused_online_no_faults": lambda: ftgemm.gemm_f64_unfused(
                h, dA, dB, dC, 1.5, 0.5, cfg=ftgemm.make_config(interval_k=kc_online)),
            "slabs_unprotected": lambda: ftgemm.gemm_f64_unfused(
                h, dA, dB, dC, 1.5, 0.5, cfg=ftgemm.make_config(abft=False, interval_k=kc_online)),
        }
        h.reset()
        t = timed_ab(torch, fns, max(2, steps // 3), 1)
        rep = h.read()
        p_mm = fl / t["unprotected"] / 1e9          # TFLOP/s
        p_mv = 2.0 / 8.0 * PEAK_HBM / 1e3           # TFLOP/s at the HBM peak
        model = lambda kk: 100.0 * (6 + 2.0 * kk) * p_mm / (n * p_mv)
        row = {"n": n, "kc_online": kc_online,
               **{f"ms_{k}": v for k, v in t.items()},
               "overhead_pct": {k: 100.0 * (v / t["unprotected"] - 1.0) for k, v in t.items()
                                if k != "unprotected"},
               "abft_passes_over_slabs_pct": 100.0 * (t["unfused_online"] / t["slabs_unprotected"] - 1.0),
               "model_overhead_pct": {"offline": model(1), "online": model(n // kc_online)},
               "faults": {"injected": rep.injected, "corrected": rep.corrected_subtract + rep.corrected_recompute,
                          "uncorrectable": rep.uncorrectable}}
        rows.append(row)
        print(json.dumps({"unfused_row": row}), file=sys.stderr, flush=True)
        del dA, dB, dC
    return rows


def dmr_routines(torch, ftgemm, h, steps):
    """The duplicated-computation routines of §4 at HBM-filling sizes: DSCAL
    (x := -x) and DNRM2 over 2^28 doubles, DGEMV without transpose and
    transposed at 16384^2 (alpha = 1, beta = 0.5), DTRSV lower at n = 16384
    (diagonal in [1, 2], off-diagonal U[-1,1] * 0.5/n; x reset before each
    solve); all U[-1,1].  Each is timed protected, protected with 20 injected
    faults per call (the paper's error-injection experiment, §6.3), and with
    protection off; GB/s count the routine's algorithmic bytes (DSCAL 16 n,
    DNRM2 8 n, DGEMV 8 (mn + n + 2m), DTRSV 8 (n(n+1)/2 + 2n)) against the
    8 TB/s HBM peak."""
    g = torch.Generator(device="cuda").manual_seed(17)
    rnd = lambda *shape: torch.rand(shape, generator=g, device="cuda", dtype=torch.float64) * 2 - 1
    out = {}

    def leg(name, nbytes, fn, calls):
        cp, cu = ftgemm.make_config(), ftgemm.make_config(abft=False)
        cf = ftgemm.make_config(seed=23, n_faults=20)
        h.reset()
        t = timed_ab(torch, {"p": lambda: fn(cp), "f": lambda: fn(cf), "u": lambda: fn(cu)}, calls, 2)
        rep = h.read()
        r = {"ms_protected": t["p"], "ms_with_20_faults": t["f"], "ms_unprotected": t["u"],
             "gbs_protected": nbytes / t["p"] / 1e6, "gbs_unprotected": nbytes / t["u"] / 1e6,
             "hbm_frac_protected": nbytes / t["p"] / 1e6 / PEAK_HBM,
             "overhead_pct": 100.0 * (t["p"] / t["u"] - 1.0),
             "overhead_with_faults_pct": 100.0 * (t["f"] / t["u"] - 1.0),
             "faults": {"injected": rep.injected, "corrected": rep.corrected_recompute,
                        "uncorrectable": rep.uncorrectable}}
        out[name] = r
        print(json.dumps({name: r}), file=sys.stderr, flush=True)

    n1 = 1 << 28
    x = rnd(n1)
    # context: what torch's own streaming kernels reach on the same 2 GiB vector
    y = torch.empty_like(x)
    t = timed_ab(torch, {"copy": lambda: y.copy_(x), "scale": lambda: x.mul_(-1.0),
                         "norm": lambda: torch.linalg.vector_norm(x)}, steps, 2)
    out["torch_reference"] = {"copy_gbs": 16.0 * n1 / t["copy"] / 1e6, "mul_inplace_gbs": 16.0 * n1 / t["scale"] / 1e6,
                              "vector_norm_gbs": 8.0 * n1 / t["norm"] / 1e6}
    print(json.dumps({"torch_reference": out["torch_reference"]}), file=sys.stderr, flush=True)
    del y
    leg("dscal_2^28", 16.0 * n1, lambda c: ftgemm.dscal_f64(h, x, -1.0, cfg=c), steps)
    res = torch.empty(1, dtype=torch.float64, device="cuda")
    leg("dnrm2_2^28", 8.0 * n1, lambda c: ftgemm.dnrm2_f64(h, x, res, cfg=c), steps)
    del x
    n2 = 16384
    A = rnd(n2, n2)
    xv, yv = rnd(n2), rnd(n2)
    for ta in (0, 1):
        leg(f"dgemv_{'t' if ta else 'n'}_{n2}", 8.0 * (n2 * n2 + 3 * n2),
            lambda c, ta=ta: ftgemm.dgemv_f64(h, A, xv, yv, 1.0, 0.5, ta, cfg=c), steps)
    A.mul_(0.5 / n2)
    A.diagonal().copy_(torch.rand(n2, generator=g, device="cuda", dtype=torch.float64) + 1.0)
    x0 = rnd(n2)
    xs = x0.clone()
    leg(f"dtrsv_{n2}", 8.0 * (n2 * (n2 + 1) / 2 + 2 * n2),
        lambda c: (xs.copy_(x0), ftgemm.dtrsv_f64(h, A, xs, ftgemm.LOWER, ftgemm.OP_N, cfg=c)), max(2, steps // 2))
    del A
    return out


def level3_routines(torch, ftgemm, h, steps, n=8192):
    """FT-DSYMM (C := 1.5 A B + 0.5 C, A symmetric lower), FT-DTRMM
    (B := 1.5 op(A) B) and FT-DTRSM (B := 1.5 op(A)^-1 B), A lower, left, no
    transpose, at m = n = 8192, U[-1,1] operands (for DTRSM a well-conditioned
    triangle: diagonal in [1, 2], off-diagonal U[-1,1] * 0.5/n), protected with
    one flip per 2^32 MACs (and without injection) against the same routine
    with ABFT off.  TFLOP/s
    count the routine's own multiply-adds: 2 m^2 n for DSYMM, m^2 n for DTRMM
    and DTRSM."""
    g = torch.Generator(device="cuda").manual_seed(11)
    rnd = lambda: torch.rand((n, n), generator=g, device="cuda", dtype=torch.float64) * 2 - 1
    A, B, C = rnd(), rnd(), rnd()
    B0 = B.clone()
    At = A * (0.5 / n)
    At.diagonal().copy_(torch.rand(n, generator=g, device="cuda", dtype=torch.float64) + 1.0)
    rate = 2.0 ** -32
    cp = ftgemm.make_config(seed=3, per_mac_rate=rate)
    cn = ftgemm.make_config()
    cu = ftgemm.make_config(abft=False)
    out = {}
    for name, fl, fn in [
        ("dsymm", 2.0 * n ** 3, lambda c: ftgemm.dsymm_f64(h, A, B0, C, 1.5, 0.5, 0, 0, c)),
        ("dtrmm", 1.0 * n ** 3, lambda c: (B.copy_(B0), ftgemm.dtrmm_f64(h, A, B, 1.5, 0, 0, 0, 0, c))),
        ("dtrsm", 1.0 * n ** 3, lambda c: (B.copy_(B0), ftgemm.dtrsm_f64(h, At, B, 1.5, 0, 0, 0, 0, c))),
    ]:
        h.reset()
        t = timed_ab(torch, {"p": lambda: fn(cp), "n": lambda: fn(cn), "u": lambda: fn(cu)},
                     max(2, steps // 2), 1)
        rep = h.read()
        out[name] = {"m": n, "n": n, "ms_protected": t["p"], "ms_protected_no_faults": t["n"],
                     "ms_unprotected": t["u"],
                     "tflops_protected": fl / t["p"] / 1e9, "tflops_unprotected": fl / t["u"] / 1e9,
                     "overhead_pct": 100.0 * (t["p"] / t["u"] - 1.0),
                     "overhead_no_faults_pct": 100.0 * (t["n"] / t["u"] - 1.0),
                     "faults": {"injected": rep.injected,
                                "corrected": rep.corrected_subtract + rep.corrected_recompute,
                                "uncorrectable": rep.uncorrectable}}
        print(json.dumps({name: out[name]}), file=sys.stderr, flush=True)
    return out


def batched_problem_seed(seed: int, p: int) -> int:
    """Injector seed of problem p of a batched call (the rule documented with
    ftg_dgemm_batched_uneven): output 2^32 + p of SplitMix64 seeded with `seed`."""
    m64 = 2 ** 64 - 1
    z = (seed + (2 ** 32 + p + 1) * 0x9E3779B97F4A7C15) & m64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m64
    return z ^ (z >> 31)


def cfg5_batched(torch, ftgemm, h, steps):
    """512 FP64 problems, m, n, k log-uniform in [32, 2048] (seed 7), alpha = 1,
    beta = 0, U[-1,1] operands, 0-2 flips per problem (U{0,1,2}, seed 7).  The
    batched call's tiles come from the autotuner (per shape bucket, timed on the
    GPU first); it runs eager and hipGraph-replayed, and against the same
    problems as 512 single protected calls (each with its own faults)."""
    from paper_2104_00897_amd import inputs, tune
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
    stream = ftgemm.current_stream_ptr
    fl = float(sum(2.0 * m * n * k for m, n, k in sizes))
    # the autotuner fills a handle's table for the batched tiles of every bucket present
    hb = ftgemm.Handle(capacity=16384)
    t0 = time.perf_counter()
    table = tune.autotune_batched(hb, sizes)
    tune_s = time.perf_counter() - t0
    picked = {t: sum(1 for m, n, k in sizes if table.get(ftgemm.F64, m, n, k) == t) for t in (2, 3)}
    cp = ftgemm.make_config(seed=7, n_faults=1)
    cu = ftgemm.make_config(abft=False)
    cp3 = ftgemm.make_config(tile=3, seed=7, n_faults=1)
    cu3 = ftgemm.make_config(abft=False, tile=3)
    # looped single calls: problem p draws from the seed the batched call gives it
    singles = [ftgemm.make_config(seed=batched_problem_seed(7, p), n_faults=int(f))
               for p, f in enumerate(faults)]

    def looped(cfgs):
        for (A, B, C), c in zip(keep, cfgs):
            ftgemm.gemm_f64(h, A, B, C, 1.0, 0.0, cfg=c)

    hb.reset()
    t = timed_ab(torch, {"p": lambda: hb.dgemm_batched(plan, stream(), cp, faults),
                         "u": lambda: hb.dgemm_batched(plan, stream(), cu),
                         "p3": lambda: hb.dgemm_batched(plan, stream(), cp3, faults),
                         "u3": lambda: hb.dgemm_batched(plan, stream(), cu3)}, steps, 2)
    rep = hb.read()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr):
        hb.dgemm_batched(plan, stream(), cp, faults)
    tg = time_calls(torch, gr.replay, steps, 2)
    torch.cuda.synchronize()
    del gr
    h.reset()
    tl = timed_ab(torch, {"p": lambda: looped(singles), "u": lambda: looped([cu] * len(keep))},
                  max(2, steps // 2), 1)
    rep_l = h.read()
    requested = int(faults.sum())
    per_call = rep.injected // (4 * (steps + 2))  # four timed runs of steps + 2 warm-up calls
    out = {"workload": "512 FP64 problems, m,n,k log-uniform [32, 2048], seed 7, 0-2 flips each",
           "gflop": fl / 1e9,
           "autotune": {"seconds": tune_s, "buckets": len(table.entries), "problems_on_tile": picked},
           "ms_protected": t["p"], "ms_unprotected": t["u"], "ms_protected_graph": tg,
           "tflops_protected": fl / t["p"] / 1e9, "tflops_unprotected": fl / t["u"] / 1e9,
           "tflops_protected_graph": fl / tg / 1e9,
           "overhead_pct": 100.0 * (t["p"] / t["u"] - 1.0),
           "fixed_tile3": {"ms_protected": t["p3"], "ms_unprotected": t["u3"],
                           "tflops_protected": fl / t["p3"] / 1e9,
                           "overhead_pct": 100.0 * (t["p3"] / t["u3"] - 1.0)},
           "looped_single_calls": {"ms_protected": tl["p"], "ms_unprotected": tl["u"],
                                   "tflops_protected": fl / tl["p"] / 1e9,
                                   "tflops_unprotected": fl / tl["u"] / 1e9,
                                   "batched_speedup_protected": tl["p"] / t["p"]},
           "faults": {"requested_per_call": requested, "injected_per_call": per_call,
                      "capped_per_call": requested - per_call,
                      "injected": rep.injected, "corrected": rep.corrected_subtract + rep.corrected_recompute,
                      "uncorrectable": rep.uncorrectable,
                      "looped_injected": rep_l.injected,
                      "looped_corrected": rep_l.corrected_subtract + rep_l.corrected_recompute}}
    hb.close()
    return out


def cpu_baseline(host, k):
    """The oracle on a bounded sample of the headline workload, on the host cores:
    its plain definition of the product (OpenMP over columns, every thread the
    process may use) on the leading 1024 x 1024 block of C with the full k, and
    its simulation of the protected procedure (one thread) on the leading
    512 x 512 block."""
    import oracle
    import platform
    A, B, C = host
    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    ms = ns = 1024
    t0 = time.perf_counter()
    oracle.gemm(np.asfortranarray(A[:ms, :]), np.asfortranarray(B[:, :ns]),
                np.asfortranarray(C[:ms, :ns]), 1.5, 0.5)
    dt = time.perf_counter() - t0
    flops = 2.0 * ms * ns * k
    ma = 512
    t1 = time.perf_counter()
    oracle.abft(np.asfortranarray(A[:ma, :]), np.asfortranarray(B[:, :ma]),
                np.asfortranarray(C[:ma, :ma]), 1.5, 0.5, bm=128, bn=128)
    da = time.perf_counter() - t1
    fa = 2.0 * ma * ma * k
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle.gemm (OpenMP, {threads} threads) on the leading {ms}x{ns} block of C "
                      f"with k={k}: {flops / 1e9:.1f} GFLOP in {dt:.1f} s",
            "host": {"cpu_model": model, "logical_cpus": os.cpu_count(), "omp_threads": threads},
            "abft_one_thread": {"value": fa / da / 1e12, "unit": "TFLOP/s", "cores": 1,
                                "sample": f"oracle.abft on the leading {ma}x{ma} block with k={k} "
                                          f"(128x128 tiles): {fa / 1e9:.1f} GFLOP in {da:.1f} s"}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2104_00897_amd import ftgemm

    if args.copy_calibration:
        a = torch.empty(2 ** 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 2 ** 30}), flush=True)
        return
    h = ftgemm.Handle(capacity=16384)
    if args.calibrate:
        print(json.dumps({"calibrate": calibrate_lambda(torch, ftgemm, h, args.calibrate)}), flush=True)
        return
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
                     "traffic": TRAFFIC_F64.get(n),
                     "kernel": f"protected FP64 product kernel (tile configuration {res['tile']})",
                     "kernel_ms": round(res["kernel_ms_protected"], 4)},
    }
    print(json.dumps({"headline": res}), file=sys.stderr, flush=True)
    if args.tiles:
        for t in (1, 2, 3, 4, 5):
            r, _ = measure(torch, ftgemm, h, n, n, n, 1.5, 0.5, 0, 0, max(3, args.steps // 2), 1, t)
            print(json.dumps({"tile_sweep": r}), file=sys.stderr, flush=True)
    if not args.no_sweep:
        sweep = []
        shapes = [(nn, nn, nn, 0) for nn in (1024, 2048, 4096, 8192) if nn != n]
        shapes += [(16384, 16384, kk, ta) for kk in (128, 256, 512) for ta in (0, 1)]
        for mm, nn, kk, ta in shapes:
            r, _ = measure(torch, ftgemm, h, mm, nn, kk, 1.5, 0.5, ta, 0, args.steps, 2, 0)
            sweep.append({key: (round(v, 4) if isinstance(v, float) else v) for key, v in r.items()})
            print(json.dumps({"sweep": r}), file=sys.stderr, flush=True)
        line["sweep"] = sweep
    if not args.no_configs:
        only = set(x for x in args.only.split(",") if x)
        cf = {}
        for name, fn in [("cfg1", lambda: cfg1_latency(torch, ftgemm, h, args.steps)),
                         ("cfg3_bf16", lambda: cfg3_lowp(torch, ftgemm, h, "bf16", args.steps,
                                                         fp_calls=args.fp_calls)),
                         ("cfg3_fp8", lambda: cfg3_lowp(torch, ftgemm, h, "fp8", args.steps,
                                                        fp_calls=args.fp_calls)),
                         ("cfg4", lambda: cfg4_ftlinear(torch, ftgemm, h, max(2, args.steps // 2))),
                         ("cfg5", lambda: cfg5_batched(torch, ftgemm, h, args.steps)),
                         ("unfused", lambda: unfused_comparison(torch, ftgemm, h, args.steps)),
                         ("level3", lambda: level3_routines(torch, ftgemm, h, args.steps)),
                         ("dmr", lambda: dmr_routines(torch, ftgemm, h, args.steps))]:
            if only and name.split("_")[0] not in only:
                continue
            cf[name] = fn()
            print(json.dumps({name: cf[name]}), file=sys.stderr, flush=True)
        line["configs"] = cf
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(host, n)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
