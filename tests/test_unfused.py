"""GPU parity of the unfused comparator (ftg_dgemm_unfused: the online ABFT of
§5.1 built around the unprotected product, whole-matrix checksums checked after
every rank-K_c update), through the C ABI, against the CPU oracle.

The oracle simulates the same procedure when its output tile is the whole
matrix (bm = m, bn = n) and its verification interval is K_c: with alpha = 1
and beta = 0 the scheme checks the accumulated product itself after every
slab, as the oracle does, so the located elements and the kinds of the
records must agree; faults planned with a 128-step granularity equal to K_c
land at slab ends, where this scheme flips them.  For general alpha and beta
the result must match the oracle's product within the rounding bound and
every injected fault must be corrected."""
import numpy as np
import pytest

import oracle
from paper_2104_00897_amd import inputs
from tests.gpu_util import assert_close_f64, check_flip_values, magnitude

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2104_00897_amd import ftgemm
    assert torch.cuda.is_available()
    h = ftgemm.Handle(capacity=4096)
    yield ftgemm, h, torch
    torch.cuda.synchronize()
    h.close()


def run(env, A, B, C, alpha, beta, ta, tb, cfg):
    ftgemm, h, torch = env
    dA, dB = ftgemm.to_device(A), ftgemm.to_device(B)
    m = A.shape[1] if ta else A.shape[0]
    n = B.shape[0] if tb else B.shape[1]
    dC = ftgemm.to_device(C) if C is not None else torch.full((n, m), float("nan"), dtype=torch.float64,
                                                               device="cuda")
    h.reset()
    ftgemm.gemm_f64_unfused(h, dA, dB, dC, alpha, beta, ta, tb, cfg=cfg)
    torch.cuda.synchronize()
    return ftgemm.to_host(dC), h.read()


def plan(seed, F, m, n, k, kc, bit_lo=52, bit_hi=62, target=oracle.TARGET_ACC):
    return oracle.fault_plan(seed, F, m, n, k, m, n, kc=kc, kgran=kc or k, bit_lo=bit_lo,
                             bit_hi=bit_hi, target=target)


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("kc", [0, 128, 256])
def test_fault_free_matches_oracle(env, ta, tb, kc):
    ftgemm = env[0]
    m, n, k = 301, 283, 397                         # ragged last slab for kc = 128, 256
    A, B, C = inputs.gemm_operands_f64(m, n, k, seed=31, ta=ta, tb=tb)
    for alpha, beta in [(1.0, 0.0), (1.5, 0.5), (-2.0, 1.0)]:
        out, rep = run(env, A, B, C if beta else None, alpha, beta, ta, tb,
                       ftgemm.make_config(interval_k=kc))
        ref = oracle.gemm(A, B, C if beta else None, alpha, beta, ta, tb)
        assert_close_f64(out, ref, magnitude(A, B, C, alpha, beta, ta, tb), k)
        assert rep.detected == 0 and rep.records == []
        assert 0.0 < rep.max_pass_ratio < 0.5


def test_integer_exact_bitwise(env):
    ftgemm = env[0]
    m, n, k = 200, 140, 384
    A, B, C = inputs.integer_operands(m, n, k, seed=32)
    out, rep = run(env, A, B, C, 1.5, -2.0, 0, 0, ftgemm.make_config(interval_k=128))
    np.testing.assert_array_equal(out, oracle.gemm(A, B, C, 1.5, -2.0))
    assert rep.detected == 0


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 1)])
def test_records_match_oracle_alpha1_beta0(env, ta, tb):
    """One flip per slab (exponent bits): located where the oracle's simulation of
    the whole-matrix scheme with interval K_c locates it, with the same kind."""
    ftgemm = env[0]
    m, n, k, kc = 260, 230, 640, 128
    A, B, _ = inputs.gemm_operands_f64(m, n, k, seed=33, ta=ta, tb=tb)
    F = k // kc
    for seed in (1, 2, 3):
        cfg = ftgemm.make_config(interval_k=kc, seed=seed, n_faults=F, bit_lo=52, bit_hi=62)
        out, rep = run(env, A, B, None, 1.0, 0.0, ta, tb, cfg)
        p = plan(seed, F, m, n, k, kc)
        got = sorted((g["row"], g["col"], g["pflip"], g["bit"]) for g in rep.inject_log)
        assert got == sorted((f.row, f.col, f.pflip, f.bit) for f in p)
        check_flip_values(rep.inject_log)
        _, orecs, ocnt = oracle.abft(A, B, None, 1.0, 0.0, ta, tb, bm=m, bn=n, kc=kc, plan=p)
        assert sorted((r["interval"], r["row"], r["col"], r["kind"]) for r in rep.records) == \
            sorted((r.interval, r.row, r.col, r.kind) for r in orecs)
        assert rep.corrected_subtract + rep.corrected_recompute == F
        ref = oracle.gemm(A, B, None, 1.0, 0.0, ta, tb)
        assert_close_f64(out, ref, magnitude(A, B, None, 1.0, 0.0, ta, tb), k)


@pytest.mark.parametrize("kc", [0, 256])
def test_faults_corrected_with_beta(env, kc):
    ftgemm = env[0]
    m, n, k = 333, 290, 768
    A, B, C = inputs.gemm_operands_f64(m, n, k, seed=34)
    F = max(1, k // kc if kc else 1)
    for bits in [(52, 62), (60, 62)]:                 # exponent flips; the second forces recomputes
        cfg = ftgemm.make_config(interval_k=kc, seed=9, n_faults=F, bit_lo=bits[0], bit_hi=bits[1])
        out, rep = run(env, A, B, C, 1.5, 0.5, 0, 0, cfg)
        assert rep.injected == F and rep.uncorrectable == 0
        assert rep.corrected_subtract + rep.corrected_recompute == F
        assert sorted((g["row"], g["col"]) for g in rep.inject_log) == \
            sorted((r["row"], r["col"]) for r in rep.records)
        ref = oracle.gemm(A, B, C, 1.5, 0.5)
        assert_close_f64(out, ref, magnitude(A, B, C, 1.5, 0.5, 0, 0), k)


def test_checksum_fault_and_two_faults(env):
    ftgemm = env[0]
    m, n, k, kc = 256, 256, 512, 128
    A, B, C = inputs.gemm_operands_f64(m, n, k, seed=35)
    cfg = ftgemm.make_config(interval_k=kc, seed=4, n_faults=4, bit_lo=52, bit_hi=62,
                             target=ftgemm.TARGET_CHECKSUM)
    out, rep = run(env, A, B, C, 1.0, 1.0, 0, 0, cfg)
    # the faulty checksum is re-based on the data, so later slabs check clean
    assert rep.injected == 4 and rep.checksum_only == 4 and rep.detected == 4
    assert all(r["kind"] == ftgemm.KIND_CHECKSUM_ONLY and r["col"] == -1 for r in rep.records)
    assert_close_f64(out, oracle.gemm(A, B, C, 1.0, 1.0), magnitude(A, B, C, 1.0, 1.0, 0, 0), k)
    cfg = ftgemm.make_config(interval_k=kc, seed=5, n_faults=2, bit_lo=56, bit_hi=62,
                             target=ftgemm.TARGET_TWO_IN_SLOT)
    out, rep = run(env, A, B, C, 1.0, 0.0, 0, 0, cfg)
    # an uncorrectable slab leaves its errors in C, so every later check flags
    # them again: the oracle's simulation of the scheme counts the same slabs
    p = plan(5, 2, m, n, k, kc, 56, 62, oracle.TARGET_TWO_IN_SLOT)
    _, orecs, ocnt = oracle.abft(A, B, None, 1.0, 0.0, bm=m, bn=n, kc=kc, plan=p)
    assert rep.injected == 4 and rep.status == ftgemm.ERR_UNCORRECTED
    assert rep.uncorrectable == ocnt["uncorrectable"] >= 2
    assert sorted(r["interval"] for r in rep.records) == sorted(r.interval for r in orecs)
