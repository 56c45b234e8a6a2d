"""GPU parity of the BF16 / FP8 protected GEMM with verification intervals
(cfg interval_k = K_c) against the CPU oracle, through the C ABI.

With intervals the product runs as rank-K_c updates of C, each checked as a
product of its own: C := alpha op(A)[:, S_t] op(B)[S_t, :] + beta_t C over the
steps S_t of interval t, beta_t = beta for the first interval and 1 after (the
K_c loop of the blocked GEMM, paper 5.1, with the per-update check of 2.1).  The
oracle simulates the same scheme (abft(..., split=True)).  Bars:
  * integer-exact inputs: every partial sum is exact in binary32, so the result
    equals the exact product bitwise, for ragged last intervals (which the wide
    tile hands to the 128 x 128 tile) and both tile configurations;
  * random inputs: within the FP32 accumulation bound, nothing flagged; one
    interval reproduces the call without intervals bitwise;
  * seeded flips: the injection log is the oracle's plan for (tile, interval)
    slots; a flip whose error clears 4 tau of its interval is located in its
    interval and corrected, with the oracle's delta, and the oracle locates it
    too; the result is then the exact product."""
import numpy as np
import pytest

import oracle
from tests.test_parity_lowp import U32, Run, assert_close32, default_lambda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2104_00897_amd import ftgemm
    assert torch.cuda.is_available()
    h = ftgemm.Handle(capacity=8192)
    yield ftgemm, h, torch
    torch.cuda.synchronize()
    h.close()


def exact(r, alpha, beta):
    a = r.va.T if r.ta else r.va
    b = r.vb.T if r.tb else r.vb
    out = r.alpha_eff(alpha) * (a @ b)
    if beta != 0:
        out = out + beta * r.C.astype(np.float64)
    return out


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
@pytest.mark.parametrize("tile", [1, 2])
@pytest.mark.parametrize("k,kc", [(700, 256), (768, 256), (700, 128)])
def test_interval_integer_exact(env, kind, tile, k, kc):
    ftgemm = env[0]
    r = Run(env, kind, 300, 270, k, 0, 0, seed=11, integer=True)
    for alpha, beta in [(1.0, 0.0), (1.5, 0.5)]:
        out, rep = r.gpu(alpha, beta, ftgemm.make_config(interval_k=kc, tile=tile))
        np.testing.assert_array_equal(out, exact(r, alpha, beta))
        assert rep.detected == 0, rep.records[:3]


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 1)])
def test_interval_random_within_bound_no_false_flags(env, kind, ta, tb):
    ftgemm = env[0]
    r = Run(env, kind, 260, 390, 1000, ta, tb, seed=12)
    for alpha, beta in [(1.0, 0.0), (1.5, 0.5)]:
        out, rep = r.gpu(alpha, beta, ftgemm.make_config(interval_k=256, tile=2))
        assert_close32(out, r.oracle(alpha, beta), r.magnitude(alpha, beta), r.k)
        assert rep.detected == 0, rep.records[:3]
    # one interval (K_c >= k) is the call without intervals
    one, _ = r.gpu(1.5, 0.5, ftgemm.make_config(interval_k=1024, tile=2))
    plain, _ = r.gpu(1.5, 0.5, ftgemm.make_config(tile=2))
    np.testing.assert_array_equal(one, plain)


def interval_taus(r, alpha, beta, kc, log):
    """Threshold of each injected element in its interval t under the binary32
    rule, the larger of its tile row's and column's: 2 lambda sqrt(k_t + len + 8)
    u32 M with M_i = |alpha| (sum_{p in S_t} |a_ip|) max_{p in S_t} sum_{j in J}
    |b_pj| + |beta_t| sum_{j in J} |C_t(i, j)|, C_t the result before interval t
    (integer operands: the exact partial product)."""
    av = r.va.T if r.ta else r.va
    bv = r.vb.T if r.tb else r.vb
    a, b = np.abs(av), np.abs(bv)
    lam = default_lambda()
    ae = abs(r.alpha_eff(alpha))
    out = []
    for g in log:
        i, j, t = g["row"], g["col"], g["interval"]
        lo, hi = t * kc, min(r.k, (t + 1) * kc)
        I = slice((i // 128) * 128, min(r.m, (i // 128) * 128 + 128))
        J = slice((j // 128) * 128, min(r.n, (j // 128) * 128 + 128))
        R, Q = I.stop - I.start, J.stop - J.start
        mr = ae * a[i, lo:hi].sum() * b[lo:hi, J].sum(axis=1).max()
        mc = ae * b[lo:hi, j].sum() * a[I, lo:hi].sum(axis=0).max()
        bt = beta if t == 0 else 1.0
        if bt != 0:
            ct = r.alpha_eff(alpha) * (av[:, :lo] @ bv[:lo, :]) + beta * r.C.astype(np.float64)
            mr += abs(bt) * np.abs(ct[i, J]).sum()
            mc += abs(bt) * np.abs(ct[I, j]).sum()
        out.append(max(oracle.tau(hi - lo + Q + 8, mr, acc32=True, lam=lam),
                       oracle.tau(hi - lo + R + 8, mc, acc32=True, lam=lam)))
    return out


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
@pytest.mark.parametrize("tile", [1, 2])
def test_interval_flips_located_and_corrected(env, kind, tile):
    ftgemm = env[0]
    k, kc, F = 700, 256, 24
    r = Run(env, kind, 530, 400, k, 0, 0, seed=13, integer=True)
    n_big = 0
    for alpha, beta in [(1.0, 0.0), (1.5, 0.5)]:
        cfg = ftgemm.make_config(interval_k=kc, tile=tile, seed=41, n_faults=F, bit_lo=24, bit_hi=30)
        out, rep = r.gpu(alpha, beta, cfg)
        plan = oracle.fault_plan(41, F, r.m, r.n, r.k, 128, 128, kc=kc, kgran=128, bit_lo=24, bit_hi=30)
        assert rep.injected == F and rep.uncorrectable == 0
        got = sorted((g["interval"], g["row"], g["col"], g["pflip"], g["bit"]) for g in rep.inject_log)
        assert got == sorted((f.interval, f.tile_m * 128 + f.row, f.tile_n * 128 + f.col, f.pflip, f.bit)
                             for f in plan)
        Cin = r.C.astype(np.float64) if beta else None
        _, orecs, _ = oracle.abft(r.va, r.vb, Cin, r.alpha_eff(alpha), beta, r.ta, r.tb, bm=128, bn=128,
                                  kc=kc, plan=plan, acc32=True, lam=default_lambda(), split=True)
        olocated = {(o.interval, o.row, o.col): o for o in orecs if o.kind in (1, 2)}
        fixed = {(g["interval"], g["row"], g["col"]): g for g in rep.records if g["kind"] in (1, 2)}
        ref = exact(r, alpha, beta)
        skip = np.zeros(ref.shape, dtype=bool)
        for g, tau in zip(rep.inject_log, interval_taus(r, alpha, beta, kc, rep.inject_log)):
            key = (g["interval"], g["row"], g["col"])
            d = abs(g["new_val"] - g["old_val"]) * abs(r.alpha_eff(alpha))
            if not np.isfinite(d) or d >= 4 * tau:
                n_big += 1
                assert key in fixed and key in olocated, (g, tau)
                gd, od = fixed[key]["delta"], olocated[key].delta
                if np.isfinite(od):
                    assert gd == pytest.approx(od, rel=1e-6, abs=tau), (g, gd, od)
            elif key not in fixed:
                ij = (g["row"], g["col"])
                assert abs(out[ij] - ref[ij]) <= d * 1.01 + 2 * (r.k + 2) * U32 * abs(ref[ij]) + tau, (g, tau)
                skip[ij] = True
        bad = (out != ref) & ~skip
        assert not bad.any(), np.argwhere(bad)[:5]
    assert n_big >= F // 2


def test_interval_checksum_target_and_errors(env):
    ftgemm, h, torch = env
    r = Run(env, "bf16", 256, 256, 512, 0, 0, seed=14, integer=True)
    cfg = ftgemm.make_config(interval_k=128, tile=2, seed=3, n_faults=6, bit_lo=25, bit_hi=30,
                             target=ftgemm.TARGET_CHECKSUM)
    out, rep = r.gpu(1.0, 1.0, cfg)
    plan = oracle.fault_plan(3, 6, r.m, r.n, r.k, 128, 128, kc=128, kgran=128, bit_lo=25, bit_hi=30,
                             target=oracle.TARGET_CHECKSUM)
    assert rep.injected == 6 and rep.checksum_only == 6
    assert sorted((g["interval"], g["row"]) for g in rep.records) == \
        sorted((f.interval, f.tile_m * 128 + f.row) for f in plan)
    np.testing.assert_array_equal(out, exact(r, 1.0, 1.0))
    # K_c must be a multiple of 128; at most 128 intervals
    dC = ftgemm.to_device(r.C)
    for kc in (100, 128 * 3 + 1):
        with pytest.raises(ftgemm.FtgError) as e:
            ftgemm.gemm_lowp(h, r.dA, r.dB, dC, 1.0, 0.0, 0, 0, r.ab, cfg=ftgemm.make_config(interval_k=kc))
        assert e.value.status == ftgemm.ERR_INVALID_ARG
    big = Run(env, "bf16", 64, 64, 128 * 129, 0, 0, seed=15, integer=True)
    dC = ftgemm.to_device(big.C)
    with pytest.raises(ftgemm.FtgError) as e:
        ftgemm.gemm_lowp(h, big.dA, big.dB, dC, 1.0, 0.0, 0, 0, big.ab, cfg=ftgemm.make_config(interval_k=128))
    assert e.value.status == ftgemm.ERR_UNSUPPORTED
    torch.cuda.synchronize()
