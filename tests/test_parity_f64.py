"""GPU parity of the FP64 protected GEMM against the CPU oracle (through the C ABI).

Fault-free results must match the oracle's plain triple loop within the
componentwise rounding bound (tests/gpu_util.py); on integer-exact inputs they
must match bitwise.  With seeded injection, every fault with a detectable
magnitude must be located at the planned element and corrected, the
injection log must reproduce the plan the oracle derives independently from
the same seed, and the records must agree with the oracle's simulation of the
same plan (oracle.abft)."""
import numpy as np
import pytest

import oracle
from paper_2104_00897_amd import inputs
from tests.gpu_util import (assert_close_f64, check_detectable_corrected, check_flip_values,
                            fp64_fault_taus, magnitude)

pytestmark = pytest.mark.gpu

TILES = {1: (256, 128), 2: (128, 128), 3: (64, 64), 4: (256, 128), 5: (128, 128)}


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2104_00897_amd import ftgemm
    assert torch.cuda.is_available()
    h = ftgemm.Handle(capacity=8192)
    yield ftgemm, h, torch
    torch.cuda.synchronize()
    h.close()


def run(env, A, B, C, alpha, beta, ta, tb, cfg=None, m=None, n=None, k=None):
    ftgemm, h, torch = env
    dA, dB = ftgemm.to_device(A), ftgemm.to_device(B)
    if C is None:
        mm = m if m is not None else (A.shape[1] if ta else A.shape[0])
        nn = n if n is not None else (B.shape[0] if tb else B.shape[1])
        dC = torch.full((nn, mm), float("nan"), dtype=torch.float64, device="cuda")
    else:
        dC = ftgemm.to_device(C)
    h.reset()
    ftgemm.gemm_f64(h, dA, dB, dC, alpha, beta, ta, tb, cfg=cfg, m=m, n=n, k=k)
    torch.cuda.synchronize()
    rep = h.read()
    return ftgemm.to_host(dC), rep


# ----------------------------------------------------------------------------- fault-free
@pytest.mark.parametrize("tile", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_fault_free_ragged(env, tile, ta, tb):
    ftgemm = env[0]
    m, n, k = 301, 283, 197          # several tiles and ragged tails in every dimension
    A, B, C = inputs.gemm_operands_f64(m, n, k, seed=1, ta=ta, tb=tb)
    for alpha, beta in [(1.0, 0.0), (1.5, 0.5), (-2.0, 1.0)]:
        cfg = ftgemm.make_config(tile=tile)
        out, rep = run(env, A, B, C if beta else None, alpha, beta, ta, tb, cfg)
        ref = oracle.gemm(A, B, C if beta else None, alpha, beta, ta, tb)
        assert_close_f64(out, ref, magnitude(A, B, C, alpha, beta, ta, tb), k)
        assert rep.detected == 0 and rep.records == [], rep.records[:3]


@pytest.mark.parametrize("tile", [1, 2, 3, 4, 5])
def test_unprotected_same_result(env, tile):
    ftgemm = env[0]
    m, n, k = 260, 130, 300
    A, B, C = inputs.gemm_operands_f64(m, n, k, seed=2)
    out, _ = run(env, A, B, C, 1.5, 0.5, 0, 0, ftgemm.make_config(abft=False, tile=tile))
    ref = oracle.gemm(A, B, C, 1.5, 0.5)
    assert_close_f64(out, ref, magnitude(A, B, C, 1.5, 0.5, 0, 0), k)


@pytest.mark.parametrize("tile", [1, 2, 3, 4, 5])
def test_integer_exact_bitwise(env, tile):
    ftgemm = env[0]
    m, n, k = 200, 140, 160
    A, B, C = inputs.integer_operands(m, n, k, seed=4)
    out, rep = run(env, A, B, C, 1.5, -2.0, 0, 0, ftgemm.make_config(tile=tile))
    np.testing.assert_array_equal(out, oracle.gemm(A, B, C, 1.5, -2.0))
    assert rep.detected == 0


def test_blas_special_cases(env):
    ftgemm, h, torch = env
    m, n, k = 70, 50, 40
    A, B, C = inputs.gemm_operands_f64(m, n, k, seed=3)
    # beta = 0: C is not read, NaN on input disappears (run() fills C with NaN)
    out, rep = run(env, A, B, None, 1.0, 0.0, 0, 0)
    assert np.isfinite(out).all()
    assert_close_f64(out, oracle.gemm(A, B), magnitude(A, B, None, 1.0, 0.0, 0, 0), k)
    # alpha = 0: C := beta C without reading A, B (NaN operands)
    An = np.full_like(A, np.nan); Bn = np.full_like(B, np.nan)
    out, _ = run(env, An, Bn, C, 0.0, 2.0, 0, 0)
    np.testing.assert_array_equal(out, 2.0 * C)
    # k = 0 with beta = 0: zeros
    out, _ = run(env, A[:, :0], B[:0, :], C, 1.0, 0.0, 0, 0, m=m, n=n, k=0)
    np.testing.assert_array_equal(out, np.zeros((m, n)))
    # quick return: m = 0 / alpha = 0 with beta = 1 leaves C untouched
    dC = ftgemm.to_device(C)
    dA, dB = ftgemm.to_device(A), ftgemm.to_device(B)
    for mm, nn, al in [(0, n, 1.0), (m, 0, 1.0), (m, n, 0.0)]:
        h.dgemm(0, 0, mm, nn, k, al, ftgemm.ptr(dA), m, ftgemm.ptr(dB), k, 1.0,
                ftgemm.ptr(dC), m, ftgemm.current_stream_ptr(), None)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ftgemm.to_host(dC), C)


def test_argument_errors(env):
    ftgemm, h, torch = env
    d = torch.zeros(64, dtype=torch.float64, device="cuda")
    p = ftgemm.ptr(d)
    cases = [((2, 0, 4, 4, 4, 4, 4, 4), 1), ((0, 7, 4, 4, 4, 4, 4, 4), 2),
             ((0, 0, -1, 4, 4, 4, 4, 4), 3), ((0, 0, 4, -1, 4, 4, 4, 4), 4),
             ((0, 0, 4, 4, -1, 4, 4, 4), 5), ((0, 0, 4, 4, 4, 3, 4, 4), 8),
             ((1, 0, 4, 4, 5, 4, 5, 4), 8), ((0, 0, 4, 4, 5, 4, 4, 4), 10),
             ((0, 1, 4, 5, 4, 4, 4, 4), 10), ((0, 0, 4, 4, 4, 4, 4, 3), 13)]
    for (ta, tb, m, n, k, lda, ldb, ldc), info in cases:
        with pytest.raises(ftgemm.FtgError) as e:
            h.dgemm(ta, tb, m, n, k, 1.0, p, lda, p, ldb, 0.0, p, ldc, None, None)
        assert e.value.status == ftgemm.ERR_INVALID_ARG and e.value.info == info
    bad = ftgemm.make_config(interval_k=100)          # not a multiple of 128
    with pytest.raises(ftgemm.FtgError) as e:
        h.dgemm(0, 0, 4, 4, 4, 1.0, p, 4, p, 4, 0.0, p, 4, None, bad)
    assert e.value.info == 20


# ----------------------------------------------------------------------------- injected faults
def plan_for(seed, F, m, n, k, tile, kc=0, bit_lo=40, bit_hi=63, target=oracle.TARGET_ACC):
    bm, bn = TILES[tile]
    return oracle.fault_plan(seed, F, m, n, k, bm, bn, kc=kc, kgran=128, bit_lo=bit_lo,
                             bit_hi=bit_hi, target=target)


def check_log_matches_plan(rep, plan, tile):
    bm, bn = TILES[tile]
    got = sorted((r["row"], r["col"], r["pflip"], r["bit"]) for r in rep.inject_log)
    want = sorted((f.tile_m * bm + f.row, -1 if f.target == oracle.TARGET_CHECKSUM else f.tile_n * bn + f.col,
                   f.pflip, f.bit) for f in plan)
    assert got == want
    check_flip_values(rep.inject_log)


def test_cfg1_256_four_faults(env):
    """256^3, alpha=1, beta=0, U[-1,1] seed 0, 4 seeded flips: all located and corrected."""
    ftgemm = env[0]
    m = n = k = 256
    A, B, _ = inputs.gemm_operands_f64(m, n, k, seed=0, with_c=False)
    ref = oracle.gemm(A, B)
    M = magnitude(A, B, None, 1.0, 0.0, 0, 0)
    for seed in range(6):
        cfg = ftgemm.make_config(tile=2, seed=seed, n_faults=4)
        out, rep = run(env, A, B, None, 1.0, 0.0, 0, 0, cfg)
        plan = plan_for(seed, 4, m, n, k, 2)
        check_log_matches_plan(rep, plan, 2)
        assert rep.injected == 4 and rep.detected == 4
        assert rep.corrected_subtract + rep.corrected_recompute == 4 and rep.uncorrectable == 0
        located = sorted((r["row"], r["col"]) for r in rep.records)
        assert located == sorted((f.tile_m * 128 + f.row, f.tile_n * 128 + f.col) for f in plan)
        assert_close_f64(out, ref, M, k)
        # the oracle's simulation of the same plan locates the same elements
        _, orecs, ocnt = oracle.abft(A, B, bm=128, bn=128, plan=plan)
        assert sorted((r.row, r.col) for r in orecs) == located
        assert ocnt["corrected_subtract"] + ocnt["corrected_recompute"] == 4


@pytest.mark.parametrize("tile", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0)])
def test_faults_every_tile_exponent_bits(env, tile, ta, tb):
    """Exponent/sign flips are always far above the threshold: 100% corrected."""
    ftgemm = env[0]
    m, n, k = 530, 390, 300
    A, B, C = inputs.gemm_operands_f64(m, n, k, seed=5, ta=ta, tb=tb)
    bm, bn = TILES[tile]
    slots = -(-m // bm) * -(-n // bn)
    F = min(slots, 12)
    cfg = ftgemm.make_config(tile=tile, seed=11 + tile, n_faults=F, bit_lo=52, bit_hi=63)
    out, rep = run(env, A, B, C, 1.5, 0.5, ta, tb, cfg)
    plan = plan_for(11 + tile, F, m, n, k, tile, bit_lo=52, bit_hi=63)
    check_log_matches_plan(rep, plan, tile)
    assert rep.injected == F
    assert rep.corrected_subtract + rep.corrected_recompute == F, rep.records
    ref = oracle.gemm(A, B, C, 1.5, 0.5, ta, tb)
    assert_close_f64(out, ref, magnitude(A, B, C, 1.5, 0.5, ta, tb), k)


@pytest.mark.parametrize("tile", [2, 3, 5])
def test_default_bit_range_detectable_faults_corrected(env, tile):
    """Bits 40..63 (A10): every fault whose error clears 4 tau of its tile row and
    column is located and corrected; any other fault that stays uncorrected is
    masked, its element within the flip's own size of the oracle."""
    ftgemm = env[0]
    m, n, k = 512, 512, 512
    A, B, C = inputs.gemm_operands_f64(m, n, k, seed=6)
    bm, bn = TILES[tile]
    F = 16
    cfg = ftgemm.make_config(tile=tile, seed=77, n_faults=F)
    out, rep = run(env, A, B, C, 1.5, 0.5, 0, 0, cfg)
    check_log_matches_plan(rep, plan_for(77, F, m, n, k, tile), tile)
    ref = oracle.gemm(A, B, C, 1.5, 0.5)
    M = magnitude(A, B, C, 1.5, 0.5, 0, 0)
    taus = fp64_fault_taus(A, B, C, 1.5, 0.5, 0, 0, rep.inject_log, bm, bn)
    big, masked_log = check_detectable_corrected(rep, taus, 1.5)
    assert big >= F // 2
    masked = np.zeros(ref.shape, dtype=bool)
    for g in masked_log:
        d = abs(g["new_val"] - g["old_val"]) * 1.5  # alpha scales the accumulator
        assert abs(out[g["row"], g["col"]] - ref[g["row"], g["col"]]) <= d * 1.01 + 1e-12 * M[g["row"], g["col"]]
        masked[g["row"], g["col"]] = True
    assert rep.injected == F and rep.uncorrectable == 0
    assert_close_f64(out, ref, M, k, skip=masked)


@pytest.mark.parametrize("tile", [2, 3, 5])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_direct_staging_all_transposes_ragged(env, tile, ta, tb):
    """Even leading dimensions and 16-byte aligned operands select the kernels that
    load full k-blocks straight into LDS; ragged edges in every dimension (the
    edge tiles and the k tail take the register path inside the same kernel).
    With beta != 0 and at most 256 tiles, tile 5's protected calls run its
    one-workgroup-per-CU kernel (C_in held in registers through the epilogue)."""
    ftgemm = env[0]
    m, n, k = 302, 286, 198
    A, B, C = inputs.gemm_operands_f64(m, n, k, seed=14, ta=ta, tb=tb)
    assert A.shape[0] % 2 == 0 and B.shape[0] % 2 == 0
    ref = oracle.gemm(A, B, C, 1.5, 0.5, ta, tb)
    M = magnitude(A, B, C, 1.5, 0.5, ta, tb)
    out, rep = run(env, A, B, C, 1.5, 0.5, ta, tb, ftgemm.make_config(tile=tile))
    assert_close_f64(out, ref, M, k)
    assert rep.detected == 0
    bm, bn = TILES[tile]
    F = min(8, -(-m // bm) * -(-n // bn))
    cfg = ftgemm.make_config(tile=tile, seed=40 + tile, n_faults=F, bit_lo=52, bit_hi=62)
    out, rep = run(env, A, B, C, 1.5, 0.5, ta, tb, cfg)
    check_log_matches_plan(rep, plan_for(40 + tile, F, m, n, k, tile, bit_lo=52, bit_hi=62), tile)
    assert rep.corrected_subtract + rep.corrected_recompute == F
    assert_close_f64(out, ref, M, k)
    # the unprotected kernel of the same configuration gives the same product
    out_u, _ = run(env, A, B, C, 1.5, 0.5, ta, tb, ftgemm.make_config(tile=tile, abft=False))
    assert_close_f64(out_u, ref, M, k)


def test_checksum_fault_is_checksum_only(env):
    ftgemm = env[0]
    m, n, k = 256, 256, 256
    A, B, C = inputs.gemm_operands_f64(m, n, k, seed=7)
    cfg = ftgemm.make_config(tile=2, seed=3, n_faults=4, bit_lo=52, bit_hi=62,
                             target=ftgemm.TARGET_CHECKSUM)
    out, rep = run(env, A, B, C, 1.0, 1.0, 0, 0, cfg)
    assert rep.injected == 4 and rep.checksum_only == 4
    assert all(r["kind"] == ftgemm.KIND_CHECKSUM_ONLY and r["col"] == -1 for r in rep.records)
    ref = oracle.gemm(A, B, C, 1.0, 1.0)
    assert_close_f64(out, ref, magnitude(A, B, C, 1.0, 1.0, 0, 0), k)


@pytest.mark.parametrize("beta", [0.0, 0.5])
def test_two_faults_in_slot(env, beta):
    ftgemm = env[0]
    m, n, k = 256, 256, 256
    A, B, C = inputs.gemm_operands_f64(m, n, k, seed=8)
    kw = dict(tile=2, seed=5, n_faults=2, bit_lo=56, bit_hi=62, target=ftgemm.TARGET_TWO_IN_SLOT)
    out, rep = run(env, A, B, C, 1.0, beta, 0, 0, ftgemm.make_config(**kw))
    assert rep.injected == 4 and rep.uncorrectable == 2
    assert rep.status == ftgemm.ERR_UNCORRECTED
    assert all(r["kind"] == ftgemm.KIND_UNCORRECTABLE for r in rep.records)
    out, rep = run(env, A, B, C, 1.0, beta, 0, 0, ftgemm.make_config(uncorrectable_policy=1, **kw))
    assert rep.uncorrectable == 2 and rep.tiles_recomputed == 2 and rep.status == ftgemm.OK
    ref = oracle.gemm(A, B, C if beta else None, 1.0, beta)
    assert_close_f64(out, ref, magnitude(A, B, C, 1.0, beta, 0, 0), k)


@pytest.mark.parametrize("tile", [2, 3, 5])
def test_interval_mode_many_faults_per_tile(env, tile):
    """Verification every 128 steps corrects one fault per (tile, interval) slot."""
    ftgemm = env[0]
    m, n, k = 200, 180, 640
    A, B, C = inputs.gemm_operands_f64(m, n, k, seed=9)
    bm, bn = TILES[tile]
    slots = -(-m // bm) * -(-n // bn) * (k // 128)
    F = slots // 2
    cfg = ftgemm.make_config(tile=tile, interval_k=128, seed=21, n_faults=F, bit_lo=52, bit_hi=62)
    out, rep = run(env, A, B, C, 1.5, 0.5, 0, 0, cfg)
    plan = plan_for(21, F, m, n, k, tile, kc=128, bit_lo=52, bit_hi=62)
    check_log_matches_plan(rep, plan, tile)
    assert rep.injected == F
    assert rep.corrected_subtract + rep.corrected_recompute == F
    got = sorted((r["interval"], r["row"], r["col"]) for r in rep.records)
    _, orecs, _ = oracle.abft(A, B, C, 1.5, 0.5, bm=bm, bn=bn, kc=128, plan=plan)
    assert got == sorted((r.interval, r.row, r.col) for r in orecs)
    ref = oracle.gemm(A, B, C, 1.5, 0.5)
    assert_close_f64(out, ref, magnitude(A, B, C, 1.5, 0.5, 0, 0), k)


@pytest.mark.parametrize("tile", [2, 3, 5])
def test_interval_checksum_faults_rebased(env, tile):
    """Interval kernels: a flipped maintained row checksum is a one-direction
    mismatch at its interval end (checksum only, data untouched), after which the
    checksum is re-based on the row's sum of the held values, so the later
    intervals of the tile pass even after flips to huge values: one record per
    fault, equal to the oracle's simulation of the plan; the data is the product."""
    ftgemm = env[0]
    m, n, k = 256, 256, 512
    A, B, C = inputs.gemm_operands_f64(m, n, k, seed=11)
    bm, bn = TILES[tile]
    slots = -(-m // bm) * -(-n // bn) * (k // 128)
    F = min(12, slots // 2)
    cfg = ftgemm.make_config(tile=tile, interval_k=128, seed=31, n_faults=F, bit_lo=52, bit_hi=62,
                             target=ftgemm.TARGET_CHECKSUM)
    out, rep = run(env, A, B, C, 1.0, 1.0, 0, 0, cfg)
    plan = plan_for(31, F, m, n, k, tile, kc=128, bit_lo=52, bit_hi=62, target=oracle.TARGET_CHECKSUM)
    _, orecs, ocnt = oracle.abft(A, B, C, 1.0, 1.0, bm=bm, bn=bn, kc=128, plan=plan)
    assert rep.injected == F == ocnt["injected"]
    assert (rep.detected, rep.checksum_only, rep.uncorrectable) == \
        (ocnt["detected"], ocnt["checksum_only"], ocnt["uncorrectable"])
    assert rep.corrected_subtract + rep.corrected_recompute == 0
    assert rep.detected == rep.checksum_only == F and rep.uncorrectable == 0
    got = sorted((r["interval"], r["tile_m"], r["tile_n"], r["row"], r["col"], r["kind"]) for r in rep.records)
    assert got == sorted((o.interval, o.tile_m, o.tile_n, o.row, o.col, o.kind) for o in orecs)
    ref = oracle.gemm(A, B, C, 1.0, 1.0)
    assert_close_f64(out, ref, magnitude(A, B, C, 1.0, 1.0, 0, 0), k)


@pytest.mark.parametrize("tile", [2, 5])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 1)])
def test_interval_two_faults_in_slot_recomputed(env, tile, ta, tb):
    """Interval kernels: two faults in one (tile, interval) slot are uncorrectable;
    under uncorrectable_policy 1 the tile restarts from its first interval, the
    intervals up to the failed one replayed without injection.  Tile 5 with even
    leading dimensions runs the direct-staged interval kernel."""
    ftgemm = env[0]
    m, n, k = 256, 256, 512
    A, B, C = inputs.gemm_operands_f64(m, n, k, seed=8, ta=ta, tb=tb)
    assert A.shape[0] % 2 == 0 and B.shape[0] % 2 == 0
    kw = dict(tile=tile, interval_k=128, seed=5, n_faults=2, bit_lo=56, bit_hi=62,
              target=ftgemm.TARGET_TWO_IN_SLOT)
    out, rep = run(env, A, B, C, 1.0, 0.5, ta, tb, ftgemm.make_config(uncorrectable_policy=1, **kw))
    assert rep.injected == 4 and rep.uncorrectable == 2 and rep.tiles_recomputed == 2
    assert rep.status == ftgemm.OK
    ref = oracle.gemm(A, B, C, 1.0, 0.5, ta, tb)
    assert_close_f64(out, ref, magnitude(A, B, C, 1.0, 0.5, ta, tb), k)


@pytest.mark.parametrize("ta,tb", [(1, 0), (0, 1)])
def test_interval_mode_direct_staging_transposed(env, ta, tb):
    """Tile 5's direct-staged interval kernel on transposed operands: one fault per
    (tile, interval) slot in half the slots, each located where the oracle's
    simulation locates it and corrected."""
    ftgemm = env[0]
    m, n, k = 300, 260, 512
    A, B, C = inputs.gemm_operands_f64(m, n, k, seed=10, ta=ta, tb=tb)
    assert A.shape[0] % 2 == 0 and B.shape[0] % 2 == 0
    slots = -(-m // 128) * -(-n // 128) * (k // 128)
    F = slots // 2
    cfg = ftgemm.make_config(tile=5, interval_k=128, seed=23, n_faults=F, bit_lo=52, bit_hi=62)
    out, rep = run(env, A, B, C, 1.5, 0.5, ta, tb, cfg)
    plan = plan_for(23, F, m, n, k, 5, kc=128, bit_lo=52, bit_hi=62)
    check_log_matches_plan(rep, plan, 5)
    assert rep.injected == F and rep.corrected_subtract + rep.corrected_recompute == F
    got = sorted((r["interval"], r["row"], r["col"]) for r in rep.records)
    _, orecs, _ = oracle.abft(A, B, C, 1.5, 0.5, ta, tb, bm=128, bn=128, kc=128, plan=plan)
    assert got == sorted((r.interval, r.row, r.col) for r in orecs)
    ref = oracle.gemm(A, B, C, 1.5, 0.5, ta, tb)
    assert_close_f64(out, ref, magnitude(A, B, C, 1.5, 0.5, ta, tb), k)


def test_deterministic_rerun(env):
    ftgemm = env[0]
    m, n, k = 300, 300, 300
    A, B, C = inputs.gemm_operands_f64(m, n, k, seed=10)
    cfg = ftgemm.make_config(tile=3, seed=99, n_faults=8)
    out1, rep1 = run(env, A, B, C, 1.0, 0.5, 0, 0, cfg)
    out2, rep2 = run(env, A, B, C, 1.0, 0.5, 0, 0, cfg)
    np.testing.assert_array_equal(out1, out2)
    key = lambda r: (r["row"], r["col"], r["kind"])
    assert sorted(map(key, rep1.records)) == sorted(map(key, rep2.records))


@pytest.mark.parametrize("tile", [2, 3, 5])
def test_recompute_in_other_waves_with_beta(env, tile):
    """Flips that the subtraction cannot undo (absorption) force the recompute
    path, which needs C_in at the element; placed in elements owned by waves
    other than the first, with beta != 0 (regression: C_in must be read before
    the owning wave stores the tile)."""
    ftgemm = env[0]
    m, n, k = 381, 276, 273
    A, B, C = inputs.gemm_operands_f64(m, n, k, seed=12)
    bm, bn = TILES[tile]
    chosen = []
    for seed in range(400):
        plan = plan_for(seed, 3, m, n, k, tile, bit_lo=60, bit_hi=62)
        if not all((f.row % bm) >= bm // 2 or (f.col % bn) >= bn // 2 for f in plan):
            continue
        _, orecs, ocnt = oracle.abft(A, B, C, 1.5, 0.5, bm=bm, bn=bn, plan=plan)
        if ocnt["corrected_recompute"] >= 1:
            chosen.append((seed, plan, orecs))
        if len(chosen) == 3:
            break
    assert len(chosen) == 3
    ref = oracle.gemm(A, B, C, 1.5, 0.5)
    M = magnitude(A, B, C, 1.5, 0.5, 0, 0)
    for seed, plan, orecs in chosen:
        cfg = ftgemm.make_config(tile=tile, seed=seed, n_faults=3, bit_lo=60, bit_hi=62)
        out, rep = run(env, A, B, C, 1.5, 0.5, 0, 0, cfg)
        check_log_matches_plan(rep, plan, tile)
        got = sorted((r["row"], r["col"], r["kind"]) for r in rep.records)
        assert got == sorted((r.row, r.col, r.kind) for r in orecs)
        assert_close_f64(out, ref, M, k)


@pytest.mark.parametrize("tile", [2, 3, 5])
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 1)])
def test_encode_pass_and_in_loop_encode_agree(env, tile, ta, tb):
    """The checksum row/column summed by the separate encode pass (default) and
    inside the k loop (encode_in_loop) locate the same faults; both match the oracle."""
    ftgemm = env[0]
    m, n, k = 333, 290, 410
    A, B, C = inputs.gemm_operands_f64(m, n, k, seed=13, ta=ta, tb=tb)
    ref = oracle.gemm(A, B, C, 1.5, 0.5, ta, tb)
    M = magnitude(A, B, C, 1.5, 0.5, ta, tb)
    got = []
    for in_loop in (False, True):
        cfg = ftgemm.make_config(tile=tile, seed=17, n_faults=6, bit_lo=52, bit_hi=62, encode_in_loop=in_loop)
        out, rep = run(env, A, B, C, 1.5, 0.5, ta, tb, cfg)
        assert rep.injected == 6 and rep.corrected_subtract + rep.corrected_recompute == 6
        assert_close_f64(out, ref, M, k)
        got.append(sorted((r["row"], r["col"], r["kind"]) for r in rep.records))
    assert got[0] == got[1]
