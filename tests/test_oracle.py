"""Pins of the CPU oracle (oracle/) against what the paper and the mathematics fix.

None of these tests uses the GPU library.  Each check compares the oracle with
something other than itself:
  * integer-exact brute force: entries in [-8, 8] make every product and sum
    exact in binary64, so the checksum relations of §2.1
    (e^T C = (e^T A) B,  C e = A (B e)) and the correction of §6.3 must hold
    bitwise, and numpy's integer matmul gives the exact product;
  * the worked example in tests/golden/worked_example.json;
  * closed forms (identity, rank-1, all-ones, alpha = 0, beta = 0 with NaN C);
  * the published first outputs of SplitMix64 seeded with 0;
  * bijectivity of the slot permutation (every slot hit exactly once);
  * rigor of the threshold: rounding alone never trips it on random data;
  * the threshold itself in closed form: all-ones operands fix every line's
    magnitude by hand (final check with beta, interval check, ragged edge
    tile, a tile next to one scaled by 10^6), and on random data it stays
    within a factor 2.2 of the textbook bound gamma_{k+q} |A||B|e;
  * single-bit flips against the IEEE 754 bit layout (exponent, sign,
    mantissa bits of binary32 and binary64).
A plausible slip in the oracle (a dropped beta term, a transposed operand, a
wrong sign in the correction, a checksum taken over the wrong index) breaks at
least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2104_00897_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")
ALPHAS = [0.0, 0.5, 1.0, 1.5, -2.0]


def exact_product(A, B, C, alpha, beta, ta, tb):
    """alpha*op(A)*op(B) + beta*C with integer matmul (exact for these inputs)."""
    a = (A.T if ta else A).astype(np.int64)
    b = (B.T if tb else B).astype(np.int64)
    prod = (a @ b).astype(np.float64)
    return alpha * prod + (beta * C if beta != 0 else 0.0)


# ----------------------------------------------------------------------------- GEMM
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (1.5, 0.5), (-2.0, 1.0), (0.5, -2.0)])
def test_gemm_integer_exact(ta, tb, alpha, beta):
    m, n, k = 37, 29, 53
    A, B, C = inputs.integer_operands(m, n, k, seed=3, ta=ta, tb=tb)
    out = oracle.gemm(A, B, C, alpha, beta, ta, tb)
    np.testing.assert_array_equal(out, exact_product(A, B, C, alpha, beta, ta, tb))


def test_gemm_special_cases():
    rng = np.random.default_rng(1)
    m, n, k = 9, 7, 9
    B = np.asfortranarray(rng.uniform(-1, 1, (k, n)))
    C = np.asfortranarray(rng.uniform(-1, 1, (m, n)))
    # A = I  =>  C = alpha B + beta C
    out = oracle.gemm(np.eye(m), B, C, 1.5, 0.5)
    np.testing.assert_array_equal(out, 1.5 * B + 0.5 * C)
    # k = 1  =>  rank-1: C_ij = alpha a_i b_j + beta c_ij
    a = np.asfortranarray(rng.uniform(-1, 1, (m, 1)))
    b = np.asfortranarray(rng.uniform(-1, 1, (1, n)))
    out = oracle.gemm(a, b, C, 2.0, -1.0)
    np.testing.assert_array_equal(out, 2.0 * (a * b) + (-1.0) * C)
    # all ones  =>  alpha k + beta c
    out = oracle.gemm(np.ones((m, 11)), np.ones((11, n)), C, 0.5, 2.0)
    np.testing.assert_array_equal(out, 0.5 * 11 + 2.0 * C)
    # alpha = 0  =>  beta C (A and B may hold anything)
    bad = np.full((m, k), np.nan, order="F")
    out = oracle.gemm(bad, np.full((k, n), np.inf, order="F"), C, 0.0, 3.0)
    np.testing.assert_array_equal(out, 3.0 * C)
    # beta = 0  =>  C is not read: NaN/Inf input disappears
    Cnan = np.full((m, n), np.nan, order="F")
    out = oracle.gemm(np.eye(m), B, Cnan, 1.0, 0.0)
    np.testing.assert_array_equal(out, B)


def test_gemm_quick_returns_and_errors():
    lib = oracle._load()
    C = np.full((3, 3), 7.0, order="F")
    A = np.ones((3, 3), order="F")
    # m = 0, n = 0, (alpha = 0 or k = 0) with beta = 1: C untouched
    for (m, n, k, al) in [(0, 3, 3, 1.0), (3, 0, 3, 1.0), (3, 3, 3, 0.0), (3, 3, 0, 1.0)]:
        info = lib.ftgo_gemm(0, 0, m, n, k, al, oracle._dptr(A), 3, oracle._dptr(A), 3, 1.0,
                             oracle._dptr(C), 3)
        assert info == 0
        assert np.all(C == 7.0)
    # BLAS argument numbering
    d = oracle._dptr(A)
    assert lib.ftgo_gemm(2, 0, 3, 3, 3, 1.0, d, 3, d, 3, 0.0, d, 3) == 1
    assert lib.ftgo_gemm(0, 5, 3, 3, 3, 1.0, d, 3, d, 3, 0.0, d, 3) == 2
    assert lib.ftgo_gemm(0, 0, -1, 3, 3, 1.0, d, 3, d, 3, 0.0, d, 3) == 3
    assert lib.ftgo_gemm(0, 0, 3, -1, 3, 1.0, d, 3, d, 3, 0.0, d, 3) == 4
    assert lib.ftgo_gemm(0, 0, 3, 3, -1, 1.0, d, 3, d, 3, 0.0, d, 3) == 5
    assert lib.ftgo_gemm(0, 0, 3, 3, 3, 1.0, d, 2, d, 3, 0.0, d, 3) == 8
    assert lib.ftgo_gemm(1, 0, 3, 3, 4, 1.0, d, 3, d, 4, 0.0, d, 3) == 8  # op(A)=A^T: lda >= k
    assert lib.ftgo_gemm(0, 0, 3, 3, 4, 1.0, d, 3, d, 3, 0.0, d, 3) == 10
    assert lib.ftgo_gemm(0, 0, 3, 3, 3, 1.0, d, 3, d, 3, 0.0, d, 2) == 13


def test_gemm_matches_numpy_float():
    # independent floating-point reference (LAPACK/BLAS matmul via numpy)
    A, B, C = inputs.gemm_operands_f64(64, 48, 80, seed=5)
    out = oracle.gemm(A, B, C, 1.5, 0.5)
    ref = 1.5 * (A @ B) + 0.5 * C
    mag = 1.5 * (np.abs(A) @ np.abs(B)) + 0.5 * np.abs(C)
    assert np.all(np.abs(out - ref) <= 2 * 80 * 2.0 ** -53 * mag * 1.01)


def test_gemm_entries_match_full():
    A, B, C = inputs.gemm_operands_f64(20, 30, 40, seed=2, ta=1, tb=1)
    full = oracle.gemm(A, B, C, -1.5, 2.0, 1, 1)
    rows = np.array([0, 19, 5, 7]); cols = np.array([0, 29, 13, 2])
    ent = oracle.gemm_entries(A, B, C, rows, cols, -1.5, 2.0, 1, 1)
    np.testing.assert_array_equal(ent, full[rows, cols])


# ----------------------------------------------------------------------------- worked example
def test_worked_example_golden():
    g = json.load(open(GOLDEN))
    A = np.array(g["A"], dtype=np.float64, order="F")
    B = np.array(g["B"], dtype=np.float64, order="F")
    C = oracle.gemm(A, B)
    np.testing.assert_array_equal(C, np.array(g["C"]))
    # the checksum relations of §2.1 on the encoded operands
    Ac = np.vstack([A, A.sum(axis=0)])
    Br = np.hstack([B, B.sum(axis=1, keepdims=True)])
    Cf = oracle.gemm(np.asfortranarray(Ac), np.asfortranarray(Br))
    np.testing.assert_array_equal(Cf[-1, :-1], g["eT_A_times_B"])
    np.testing.assert_array_equal(Cf[:-1, -1], g["A_times_B_e"])
    np.testing.assert_array_equal(A.sum(axis=0), g["eT_A"])
    np.testing.assert_array_equal(B.sum(axis=1), g["B_e"])
    # the flip of the example and the resulting checksum differences
    f = g["fault"]
    assert oracle.flip64(C[f["row"], f["col"]], f["bit"]) == f["faulty_value"]
    for fl in g["flips"]:
        y = oracle.flip64(fl["x"], fl["bit"])
        if fl["y"] == "inf":
            assert y == math.inf
        elif fl["y"] == "nan":
            assert math.isnan(y)
        else:
            assert y == fl["y"]
        if "delta" in fl:
            assert y - fl["x"] == fl["delta"]


def test_worked_example_abft_locates_and_corrects():
    g = json.load(open(GOLDEN))
    A = np.array(g["A"], dtype=np.float64, order="F")
    B = np.array(g["B"], dtype=np.float64, order="F")
    f = g["fault"]
    # flip after the last step (k = 2): the accumulator holds the final 10.0
    plan = [oracle.Fault(0, 0, 0, f["row"], f["col"], 1, f["bit"], oracle.TARGET_ACC)]
    C, recs, cnt = oracle.abft(A, B, bm=4, bn=4, plan=plan)
    np.testing.assert_array_equal(C, np.array(g["C"]))
    assert cnt["injected"] == 1 and cnt["detected"] == 1 and cnt["corrected_subtract"] == 1
    assert len(recs) == 1
    r = recs[0]
    assert (r.row, r.col, r.kind) == (f["row"], f["col"], oracle.KIND_SUBTRACT)
    assert r.delta == f["delta_rows"][f["row"]] == f["delta_cols"][f["col"]]
    # flip after step 0: 3*2 = 6 -> 3, then + 4*1 = 7, so delta = -3
    plan = [oracle.Fault(0, 0, 0, f["row"], f["col"], 0, f["bit"], oracle.TARGET_ACC)]
    C, recs, cnt = oracle.abft(A, B, bm=4, bn=4, plan=plan)
    np.testing.assert_array_equal(C, np.array(g["C"]))
    assert recs[0].delta == -3.0
    # sign flip of the final value: delta = -20
    plan = [oracle.Fault(0, 0, 0, f["row"], f["col"], 1, 63, oracle.TARGET_ACC)]
    C, recs, cnt = oracle.abft(A, B, bm=4, bn=4, plan=plan)
    np.testing.assert_array_equal(C, np.array(g["C"]))
    assert recs[0].delta == -20.0 and recs[0].kind == oracle.KIND_SUBTRACT


# ----------------------------------------------------------------------------- ABFT, integer exact
@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (1.5, 0.5), (-2.0, 1.0), (0.5, 1.5)])
def test_abft_fault_free_integer_exact(ta, tb, alpha, beta):
    m, n, k = 45, 38, 40
    A, B, C = inputs.integer_operands(m, n, k, seed=7, ta=ta, tb=tb)
    out, recs, cnt = oracle.abft(A, B, C, alpha, beta, ta, tb, bm=16, bn=16, kc=16)
    np.testing.assert_array_equal(out, exact_product(A, B, C, alpha, beta, ta, tb))
    assert recs == [] and cnt["detected"] == 0


@pytest.mark.parametrize("kc", [0, 16])
def test_abft_integer_faults_corrected_bitwise(kc):
    m, n, k = 48, 40, 64
    A, B, C = inputs.integer_operands(m, n, k, seed=11)
    # mantissa/exponent bits whose flips keep integers exactly representable
    plan = oracle.fault_plan(seed=5, n_faults=6, m=m, n=n, k=k, bm=16, bn=16, kc=kc, kgran=4,
                             bit_lo=50, bit_hi=53)
    assert len(plan) == 6
    out, recs, cnt = oracle.abft(A, B, C, 1.5, 0.5, bm=16, bn=16, kc=kc, plan=plan)
    np.testing.assert_array_equal(out, exact_product(A, B, C, 1.5, 0.5, 0, 0))
    assert cnt["injected"] == 6
    located = {(r.row, r.col) for r in recs if r.kind in (1, 2)}
    # a flip can be masked only if it leaves the value unchanged (never for a
    # single-bit flip), so each fault is found at its planned global position
    want = {(f.tile_m * 16 + f.row, f.tile_n * 16 + f.col) for f in plan}
    assert located == want
    assert cnt["corrected_subtract"] + cnt["corrected_recompute"] == 6
    assert cnt["uncorrectable"] == 0 and cnt["checksum_only"] == 0


# ----------------------------------------------------------------------------- correction paths
def _rand(m, n, k, seed=0, beta_c=True):
    return inputs.gemm_operands_f64(m, n, k, seed=seed, with_c=beta_c)


def _within(out, ref, A, B, C, alpha, beta, k, tol=None):
    mag = abs(alpha) * (np.abs(A) @ np.abs(B)) + (abs(beta) * np.abs(C) if beta else 0.0)
    tol = tol if tol is not None else max(1e-12, 2.2 * k * 2.0 ** -53)
    return np.all(np.abs(out - ref) <= tol * mag + 1e-300)


def test_recompute_path_for_absorbing_exponent_flip():
    m, n, k = 32, 32, 64
    A, B, C = _rand(m, n, k, seed=1)
    ref = oracle.gemm(A, B, C, 1.0, 0.0)
    # flip the top exponent bit early: the value becomes ~1e307 and absorbs later
    # updates, so subtracting delta cannot restore it (the recompute fallback must)
    plan = [oracle.Fault(0, 0, 0, 3, 5, 0, 62, oracle.TARGET_ACC)]
    out, recs, cnt = oracle.abft(A, B, C, 1.0, 0.0, bm=32, bn=32, plan=plan)
    assert [(r.row, r.col, r.kind) for r in recs] == [(3, 5, oracle.KIND_RECOMPUTE)]
    assert _within(out, ref, A, B, C, 1.0, 0.0, k)


def test_recompute_path_for_inf_and_nan():
    m, n, k = 24, 20, 16
    A = np.asfortranarray(np.full((m, k), 0.25))
    B = np.asfortranarray(np.full((k, n), 0.25))   # acc after step 0 = 0.0625 = 2^-4
    ref = oracle.gemm(A, B)
    for bit in (62,):                               # 2^-4 with bit 62 -> 2^1020 (finite, huge)
        plan = [oracle.Fault(0, 0, 0, 2, 3, 0, bit, oracle.TARGET_ACC)]
        out, recs, _ = oracle.abft(A, B, bm=32, bn=32, plan=plan)
        np.testing.assert_array_equal(out, ref)
    # acc = 1.0 at step 15 -> +Inf; acc = 1.5 is impossible here, use a NaN-producing case below
    plan = [oracle.Fault(0, 0, 0, 2, 3, 15, 62, oracle.TARGET_ACC)]
    out, recs, _ = oracle.abft(A, B, bm=32, bn=32, plan=plan)
    assert math.isinf(oracle.flip64(1.0, 62))
    np.testing.assert_array_equal(out, ref)
    assert recs[0].kind == oracle.KIND_RECOMPUTE and not math.isfinite(recs[0].delta)
    A2 = np.asfortranarray(np.full((m, 1), 1.5)); B2 = np.asfortranarray(np.ones((1, n)))
    plan = [oracle.Fault(0, 0, 0, 0, 0, 0, 62, oracle.TARGET_ACC)]   # 1.5 -> NaN
    out, recs, _ = oracle.abft(A2, B2, bm=32, bn=32, plan=plan)
    np.testing.assert_array_equal(out, oracle.gemm(A2, B2))
    assert recs[0].kind == oracle.KIND_RECOMPUTE and math.isnan(recs[0].delta)


def test_checksum_only_fault_leaves_data():
    m, n, k = 40, 40, 48
    A, B, C = inputs.integer_operands(m, n, k, seed=4)
    plan = oracle.fault_plan(seed=9, n_faults=3, m=m, n=n, k=k, bm=16, bn=16, kc=16, kgran=4,
                             bit_lo=50, bit_hi=53, target=oracle.TARGET_CHECKSUM)
    out, recs, cnt = oracle.abft(A, B, C, 1.0, 1.0, bm=16, bn=16, kc=16, plan=plan)
    np.testing.assert_array_equal(out, exact_product(A, B, C, 1.0, 1.0, 0, 0))
    assert cnt["checksum_only"] == 3 and cnt["corrected_subtract"] == 0
    assert all(r.kind == oracle.KIND_CHECKSUM_ONLY and r.col == -1 for r in recs)
    # a corrupted checksum is re-based, so no later interval of its tile flags again
    assert cnt["detected"] == 3


def test_checksum_rebased_after_huge_flip():
    """A flip of the top exponent bit makes the maintained checksum huge; the
    re-based checksum is the data's line sum, so the later intervals of the tile
    pass (adding the mismatch to the huge value would have lost the checksum's
    own value).  Data exact, one record."""
    m, n, k = 16, 16, 64
    A, B, C = inputs.integer_operands(m, n, k, seed=5)
    for bit in (62, 61, 58):
        plan = [oracle.Fault(0, 0, 0, 3, 0, 7, bit, oracle.TARGET_CHECKSUM)]
        out, recs, cnt = oracle.abft(A, B, C, 1.0, 1.0, bm=16, bn=16, kc=16, plan=plan)
        np.testing.assert_array_equal(out, exact_product(A, B, C, 1.0, 1.0, 0, 0))
        assert cnt["detected"] == 1 and cnt["checksum_only"] == 1 and cnt["uncorrectable"] == 0
        assert [(r.interval, r.row, r.col, r.kind) for r in recs] == [(0, 3, -1, oracle.KIND_CHECKSUM_ONLY)]


def test_two_faults_in_one_slot_uncorrectable():
    m, n, k = 32, 32, 32
    A, B, C = inputs.integer_operands(m, n, k, seed=6)
    plan = oracle.fault_plan(seed=2, n_faults=1, m=m, n=n, k=k, bm=32, bn=32, kgran=4,
                             bit_lo=50, bit_hi=53, target=oracle.TARGET_TWO_IN_SLOT)
    assert len(plan) == 2 and plan[0].row != plan[1].row and plan[0].col != plan[1].col
    exact = exact_product(A, B, C, 1.0, 0.0, 0, 0)
    out, recs, cnt = oracle.abft(A, B, C, 1.0, 0.0, bm=32, bn=32, plan=plan)
    assert cnt["uncorrectable"] == 1 and recs[0].kind == oracle.KIND_UNCORRECTABLE
    assert np.sum(out != exact) == 2          # reported, data left as computed
    out, recs, cnt = oracle.abft(A, B, C, 1.0, 0.0, bm=32, bn=32, plan=plan,
                                 uncorrectable_policy=1)
    assert recs[0].kind == oracle.KIND_TILE_RECOMPUTED and cnt["tiles_recomputed"] == 1
    np.testing.assert_array_equal(out, exact)


def test_interval_mode_corrects_one_fault_per_interval():
    # three faults in one tile, each in a different interval: all corrected (§2.1)
    m, n, k = 16, 16, 96
    A, B, C = inputs.integer_operands(m, n, k, seed=8)
    plan = [oracle.Fault(0, 0, t, 2 + t, 5 + 2 * t, 32 * t + 7, 51, oracle.TARGET_ACC)
            for t in range(3)]
    out, recs, cnt = oracle.abft(A, B, C, 1.0, 0.0, bm=16, bn=16, kc=32, plan=plan)
    np.testing.assert_array_equal(out, exact_product(A, B, C, 1.0, 0.0, 0, 0))
    assert [(r.interval, r.row, r.col) for r in recs] == [(t, 2 + t, 5 + 2 * t) for t in range(3)]
    # the same three faults without interval checks land in one slot: uncorrectable
    out, recs, cnt = oracle.abft(A, B, C, 1.0, 0.0, bm=16, bn=16, kc=0, plan=[
        oracle.Fault(0, 0, 0, f.row, f.col, f.pflip, f.bit, f.target) for f in plan])
    assert cnt["uncorrectable"] == 1


def test_correct_policy_always_recompute():
    A, B, C = inputs.integer_operands(20, 20, 20, seed=1)
    plan = [oracle.Fault(0, 0, 0, 4, 6, 10, 52, oracle.TARGET_ACC)]
    out, recs, _ = oracle.abft(A, B, C, 1.0, 0.0, bm=32, bn=32, plan=plan, correct_policy=1)
    np.testing.assert_array_equal(out, exact_product(A, B, C, 1.0, 0.0, 0, 0))
    assert recs[0].kind == oracle.KIND_RECOMPUTE


# ----------------------------------------------------------------------------- threshold rigor
@pytest.mark.parametrize("shape,tile,kc,ab", [
    ((128, 96, 256), (64, 32), 0, (1.5, 0.5)),
    ((100, 70, 300), (32, 64), 64, (1.0, 0.0)),
    ((64, 64, 512), (64, 64), 128, (-2.0, 1.0)),
])
def test_no_false_positive_fp64(shape, tile, kc, ab):
    m, n, k = shape
    for seed in range(3):
        A, B, C = _rand(m, n, k, seed=seed)
        out, recs, cnt = oracle.abft(A, B, C, ab[0], ab[1], bm=tile[0], bn=tile[1], kc=kc)
        assert cnt["detected"] == 0, recs
        ref = oracle.gemm(A, B, C, ab[0], ab[1])
        np.testing.assert_array_equal(out, ref)   # same order of every sum as the plain loop


def test_threshold_definition_values():
    # gamma(n) = n u / (1 - n u) with u = 2^-53 (standard model of binary64)
    for nterms in (1, 100, 4096, 16384):
        u = 2.0 ** -53
        assert oracle.gamma(nterms) == pytest.approx(nterms * u / (1 - nterms * u), rel=1e-15)
    # a fault of magnitude >= 4 tau is always flagged: tau grows linearly with the magnitude
    assert oracle.tau(1000, 2.0) == pytest.approx(2 * oracle.tau(1000, 1.0))


# ----------------------------------------------------------------------------- injector plan
def test_splitmix64_published_values():
    # first three outputs of SplitMix64 started from state 0
    assert oracle.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert oracle.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    assert oracle.splitmix64(0, 2) == 0x06C45D188009454F


@pytest.mark.parametrize("S", list(range(1, 60)) + [64, 97, 128, 1000, 4096])
def test_slot_permutation_is_bijection(S):
    a, b = oracle.slot_permutation(12345 + S, S)
    assert math.gcd(a, S) == 1 or S == 1
    assert sorted((a * r + b) % S for r in range(S)) == list(range(S))


def test_fault_plan_deterministic_distinct_capped():
    kw = dict(m=300, n=260, k=256, bm=128, bn=128, kc=64, kgran=16)
    p1 = oracle.fault_plan(seed=42, n_faults=20, **kw)
    p2 = oracle.fault_plan(seed=42, n_faults=20, **kw)
    assert p1 == p2
    slots = {(f.tile_m, f.tile_n, f.interval) for f in p1}
    assert len(slots) == len(p1) == 20
    for f in p1:
        rows = min(128, 300 - 128 * f.tile_m); cols = min(128, 260 - 128 * f.tile_n)
        assert 0 <= f.row < rows and 0 <= f.col < cols and 40 <= f.bit <= 63
        lo, hi = 64 * f.interval, 64 * f.interval + 64
        assert lo <= f.pflip < hi and (f.pflip + 1) % 16 == 0
    # capped at the number of slots: 3 x 3 tiles x 4 intervals = 36
    full = oracle.fault_plan(seed=1, n_faults=1000, **kw)
    assert len(full) == 36
    assert {(f.tile_m, f.tile_n, f.interval) for f in full} == {
        (a, b, c) for a in range(3) for b in range(3) for c in range(4)}
    assert oracle.fault_plan(seed=43, n_faults=20, **kw) != p1


# ----------------------------------------------------------------------------- binary32 threshold
def _single_fault_record(A, B, alpha, bm, bn, bit=62, lam=1.0):
    """One exponent flip (always far above any threshold) in tile (0, 0); acc32 path."""
    m, k = A.shape
    n = B.shape[1]
    plan = [oracle.Fault(0, 0, 0, 3, 5, k - 1, bit, oracle.TARGET_ACC)]
    _, recs, cnt = oracle.abft(A, B, None, alpha, 0.0, bm=bm, bn=bn, plan=plan, acc32=True, lam=lam)
    assert cnt["detected"] == 1 and len(recs) == 1
    return recs[0], min(bm, m), min(bn, n)


def test_acc32_threshold_equals_exact_magnitude_for_constant_panel_sums():
    """With B all ones every step has the same panel sum Q, so the binary32 bound
    (sum_p |a_ip|) max_p (sum_j |b_pj|) equals the exact magnitude
    sum_p |a_ip| sum_j |b_pj| = Q sum_p |a_ip|: tau follows in closed form."""
    rng = np.random.default_rng(41)
    m, n, k = 40, 24, 33
    A = np.asfortranarray(rng.uniform(-1, 1, size=(m, k)))
    B = np.ones((k, n), order="F")
    rec, R, Q = _single_fault_record(A, B, 1.5, 32, 16, bit=30, lam=2.0)
    assert (rec.row, rec.col) == (3, 5)
    mag = 1.5 * Q * np.abs(A[3, :]).sum()
    want = 2.0 * 2.0 * math.sqrt(k + Q + 8) * 2.0 ** -24 * mag * (1 + 2.0 ** -20)
    assert rec.tau == pytest.approx(want, rel=1e-12)


def test_acc32_threshold_bounds_exact_magnitude():
    """Hoelder: the binary32 bound is never below the exact magnitude of the row."""
    rng = np.random.default_rng(42)
    m, n, k = 50, 45, 70
    A = np.asfortranarray(rng.standard_normal((m, k)))
    B = np.asfortranarray(rng.standard_normal((k, n)) * np.linspace(0.1, 3, k)[:, None])
    rec, R, Q = _single_fault_record(A, B, 1.0, 32, 32, bit=30)
    exact = (np.abs(A[3, :]) * np.abs(B[:, :Q]).sum(axis=1)).sum()
    tau_exact = 2.0 * math.sqrt(k + Q + 8) * 2.0 ** -24 * exact * (1 + 2.0 ** -20)
    assert rec.tau >= tau_exact
    # and it is the Hoelder bound itself
    bound = np.abs(A[3, :]).sum() * np.abs(B[:, :Q]).sum(axis=1).max()
    assert rec.tau == pytest.approx(tau_exact * bound / exact, rel=1e-12)


def test_acc32_absorbing_flip_recomputed_small_flip_subtracted():
    """Binary32 path: a flip that lifts the value far above its row's scale has
    absorbed the true value, so the element is recomputed (and equals the
    product); a flip of a low exponent bit keeps it and is subtracted.  Either
    way the result matches numpy's product of the same operands."""
    rng = np.random.default_rng(43)
    m, n, k = 64, 48, 100
    A = np.asfortranarray(rng.standard_normal((m, k)))
    B = np.asfortranarray(rng.standard_normal((k, n)))
    ref = A @ B
    for bit, kind in [(29, oracle.KIND_RECOMPUTE), (24, oracle.KIND_SUBTRACT)]:
        plan = [oracle.Fault(0, 0, 0, 7, 9, k - 1, bit, oracle.TARGET_ACC)]
        x = float(np.float32(ref[7, 9]))
        flipped = oracle.flip32(x, bit)
        assert abs(flipped) > 1e3 * abs(x) if bit == 29 else abs(flipped) < 1e3 * abs(x) + 1
        C, recs, cnt = oracle.abft(A, B, bm=64, bn=48, plan=plan, acc32=True, lam=4.0)
        assert [(r.row, r.col, r.kind) for r in recs] == [(7, 9, kind)]
        np.testing.assert_allclose(C, ref, rtol=0, atol=1e-9 * np.abs(A).sum(axis=1).max() * np.abs(B).max())


# ----------------------------------------------------------------------------- split intervals
def _np_flip32(x, bit):
    """IEEE binary32 bit flip by the bit layout (numpy view), independent of the oracle."""
    u = np.array([x], dtype=np.float32).view(np.uint32)
    u ^= np.uint32(1 << bit)
    return float(u.view(np.float32)[0])


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 1)])
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (1.5, 0.5), (-2.0, 1.0)])
def test_split_intervals_integer_exact(ta, tb, alpha, beta):
    """C as the accumulator across K_c intervals (each interval its own product,
    beta only on the first): with no fault the result is the exact product,
    nothing is flagged, and one interval reproduces the unsplit call bitwise."""
    m, n, k = 37, 29, 50
    A, B, C = inputs.integer_operands(m, n, k, seed=21, ta=ta, tb=tb)
    exact = exact_product(A, B, C, alpha, beta, ta, tb)
    for kc in (16, 32, 48):
        out, recs, cnt = oracle.abft(A, B, C, alpha, beta, ta, tb, bm=16, bn=16, kc=kc, acc32=True,
                                     lam=4.0, split=True)
        np.testing.assert_array_equal(out, exact)
        assert cnt["detected"] == 0 and not recs
    one, _, _ = oracle.abft(A, B, C, alpha, beta, ta, tb, bm=16, bn=16, kc=0, acc32=True, lam=4.0,
                            split=True)
    ref, _, _ = oracle.abft(A, B, C, alpha, beta, ta, tb, bm=16, bn=16, kc=0, acc32=True, lam=4.0)
    np.testing.assert_array_equal(one, ref)


def test_split_delta_is_the_flip_of_the_interval_partial_sum():
    """A flip of the accumulator after step p of interval t changes the element by
    flip(s) - s with s the interval's own partial sum a_i[plo..p] . b_j[plo..p]
    (split), but the running sum over [0, p] in the online scheme, unscaled
    before the final check.  Partial sums are small integers here, so both are
    exact; each fault is located in its interval and corrected bitwise."""
    m, n, k, kc = 16, 16, 96, 32
    A, B, C = inputs.integer_operands(m, n, k, seed=8)
    alpha, beta = 1.5, 0.5
    plan = [oracle.Fault(0, 0, t, 2 + t, 5 + 2 * t, kc * t + 9 + 5 * t, 23, oracle.TARGET_ACC)
            for t in range(3)]
    for split in (True, False):
        out, recs, cnt = oracle.abft(A, B, C, alpha, beta, bm=16, bn=16, kc=kc, plan=plan, acc32=True,
                                     lam=4.0, split=split)
        np.testing.assert_array_equal(out, exact_product(A, B, C, alpha, beta, 0, 0))
        assert [(r.interval, r.row, r.col) for r in recs] == [(f.interval, f.row, f.col) for f in plan]
        for f, r in zip(plan, recs):
            lo = kc * f.interval if split else 0
            s = float(A[f.row, lo:f.pflip + 1] @ B[lo:f.pflip + 1, f.col])
            assert s != 0.0
            scale = alpha if (split or f.interval == 2) else 1.0
            assert r.delta == scale * (_np_flip32(s, 23) - s), (split, f, r)
            assert r.kind == oracle.KIND_SUBTRACT


def test_split_threshold_closed_form():
    """All-ones operands and C: interval 1 of a split call checks
    alpha A_1 B_1 + 1 C_1 with C_1 = alpha kc + beta left by interval 0, so the
    row bound is |alpha| kc Q + Q (alpha kc + beta) over kc + Q + 8 terms."""
    m, n, k, kc, lam = 32, 16, 48, 16, 2.0
    A = np.ones((m, k), order="F")
    B = np.ones((k, n), order="F")
    C = np.ones((m, n), order="F")
    alpha, beta = 2.0, 0.5
    plan = [oracle.Fault(0, 0, 1, 4, 7, 2 * kc - 1, 30, oracle.TARGET_ACC)]
    out, recs, cnt = oracle.abft(A, B, C, alpha, beta, bm=32, bn=16, kc=kc, plan=plan, acc32=True,
                                 lam=lam, split=True)
    assert cnt["detected"] == 1 and recs[0].interval == 1 and (recs[0].row, recs[0].col) == (4, 7)
    Q = 16
    M = alpha * kc * Q + Q * (alpha * kc + beta)
    want = 2.0 * lam * math.sqrt(kc + Q + 8) * 2.0 ** -24 * M * (1 + 2.0 ** -20)
    assert recs[0].tau == pytest.approx(want, rel=1e-12)
    np.testing.assert_array_equal(out, alpha * k * np.ones((m, n)) + beta)


# ----------------------------------------------------------------------------- FP64 threshold, closed form
U64 = 2.0 ** -53


def _gamma_closed(nterms):
    # the standard-model constant gamma(n) = n u / (1 - n u) of binary64
    return nterms * U64 / (1.0 - nterms * U64)


def test_fp64_threshold_closed_form_all_ones():
    """All-ones operands fix the row magnitude by hand: for a row i of tile (0,0)
    with Q columns, M_i = |alpha| k Q + |beta| Q c (c the constant C_in), and the
    final check sums k + Q terms.  The record of an exponent flip (always far
    above the threshold) must carry tau = 2 gamma(k + Q + 8) M_i (1 + 2^-20): a
    tau taken over the whole matrix, with a wrong term count, or without the beta
    term fails the equality.  The rows of A in tile (1, 0) are scaled by 10^6,
    which a tile-local magnitude never sees."""
    m, n, k = 40, 24, 33
    bm, bn = 32, 16
    A = np.ones((m, k), order="F")
    A[bm:, :] = 1e6
    B = np.ones((k, n), order="F")
    C = np.full((m, n), 0.75, order="F")
    alpha, beta = 1.5, -0.5
    plan = [oracle.Fault(0, 0, 0, 3, 5, k - 1, 62, oracle.TARGET_ACC)]
    _, recs, cnt = oracle.abft(A, B, C, alpha, beta, bm=bm, bn=bn, plan=plan)
    assert cnt["detected"] == 1 and len(recs) == 1
    Q = bn
    M = abs(alpha) * k * Q + abs(beta) * Q * 0.75
    want = 2.0 * _gamma_closed(k + Q + 8) * M * (1 + 2.0 ** -20)
    assert (recs[0].row, recs[0].col) == (3, 5)
    assert recs[0].tau == want
    # the ragged edge tile (1, 1): 8 rows of A scaled by 10^6, Q = 8 columns
    plan = [oracle.Fault(1, 1, 0, 2, 6, k - 1, 62, oracle.TARGET_ACC)]
    _, recs, cnt = oracle.abft(A, B, C, alpha, beta, bm=bm, bn=bn, plan=plan)
    Q1 = n - bn
    M1 = abs(alpha) * 1e6 * k * Q1 + abs(beta) * Q1 * 0.75
    assert cnt["detected"] == 1
    assert (recs[0].row, recs[0].col) == (bm + 2, bn + 6)
    assert recs[0].tau == 2.0 * _gamma_closed(k + Q1 + 8) * M1 * (1 + 2.0 ** -20)


def test_fp64_threshold_closed_form_interval():
    """Interval mode: a check after steps [0, p_end) compares the held accumulator
    (alpha = 1, beta = 0 mid-way), so for all-ones operands M_i = p_end Q and the
    term count is p_end + Q + 8."""
    m, n, k, kc = 32, 16, 48, 16
    A = np.ones((m, k), order="F")
    B = np.ones((k, n), order="F")
    plan = [oracle.Fault(0, 0, 1, 4, 7, 2 * kc - 1, 62, oracle.TARGET_ACC)]
    _, recs, cnt = oracle.abft(A, B, None, 2.0, 0.0, bm=32, bn=16, kc=kc, plan=plan)
    assert cnt["detected"] == 1 and recs[0].interval == 1
    p_end, Q = 2 * kc, 16
    assert recs[0].tau == 2.0 * _gamma_closed(p_end + Q + 8) * (p_end * Q) * (1 + 2.0 ** -20)


def test_fp64_threshold_within_factor_of_rigorous_bound():
    """Upper pin: tau must not exceed a small multiple of the textbook bound
    gamma_{k+Q} |alpha| |A_i| |B_J| e for random data (a tau inflated by a wrong
    term count or a magnitude over the whole matrix would be 10-100x larger)."""
    rng = np.random.default_rng(5)
    m, n, k = 96, 64, 200
    A = np.asfortranarray(rng.uniform(-1, 1, (m, k)))
    B = np.asfortranarray(rng.uniform(-1, 1, (k, n)))
    plan = [oracle.Fault(1, 1, 0, 5, 9, k - 1, 62, oracle.TARGET_ACC)]
    _, recs, cnt = oracle.abft(A, B, None, 1.0, 0.0, bm=48, bn=32, plan=plan)
    i, J = 48 + 5, slice(32, 64)
    M = float((np.abs(A[i, :]) * np.abs(B[:, J]).sum(axis=1)).sum())
    textbook = _gamma_closed(k + 32) * M
    assert textbook < recs[0].tau <= 2.2 * textbook


# ----------------------------------------------------------------------------- bit flips
@pytest.mark.parametrize("x,bit,want", [
    (1.0, 23, 0.5),            # lowest exponent bit: 0x3F800000 -> 0x3F000000
    (1.0, 31, -1.0),           # sign
    (1.0, 22, 1.5),            # top mantissa bit
    (1.0, 0, 1.0 + 2.0 ** -23),  # lowest mantissa bit
    (1.0, 30, float("inf")),   # top exponent bit: 0x7F800000
    (3.0, 24, 12.0),           # 0x40400000 -> 0x41400000: exponent 128 -> 130
])
def test_flip32_bit_patterns(x, bit, want):
    assert oracle.flip32(x, bit) == want
    assert oracle.flip32(oracle.flip32(x, bit), bit) == x


@pytest.mark.parametrize("x,bit,want", [
    (1.0, 52, 0.5), (1.0, 63, -1.0), (1.0, 51, 1.5), (1.0, 0, 1.0 + 2.0 ** -52),
    (1.0, 62, float("inf")), (10.0, 52, 20.0),
])
def test_flip64_bit_patterns(x, bit, want):
    assert oracle.flip64(x, bit) == want
    assert oracle.flip64(oracle.flip64(x, bit), bit) == x


# ----------------------------------------------------------------------------- DSYMM / DTRMM
def _sym_full(A, uplo):
    L = np.tril(A) if uplo == 0 else np.triu(A)
    return L + (L.T - np.diag(np.diag(L)))


@pytest.mark.parametrize("side,uplo", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_dsymm_integer_exact(side, uplo):
    """Only the referenced triangle is read: the other one holds NaN; the result
    equals the exact integer product with the symmetric matrix built by hand."""
    rng = np.random.default_rng(50 + side * 2 + uplo)
    m, n = 23, 17
    k = m if side == 0 else n
    A = rng.integers(-8, 9, size=(k, k)).astype(np.float64)
    full = _sym_full(A, uplo)
    Anan = A.copy()
    Anan[np.triu_indices(k, 1) if uplo == 0 else np.tril_indices(k, -1)] = np.nan
    B = rng.integers(-8, 9, size=(m, n)).astype(np.float64)
    C = rng.integers(-8, 9, size=(m, n)).astype(np.float64)
    out = oracle.dsymm(np.asfortranarray(Anan), B, C, 1.5, -2.0, side, uplo)
    fi, bi = full.astype(np.int64), B.astype(np.int64)
    prod = (fi @ bi if side == 0 else bi @ fi).astype(np.float64)
    np.testing.assert_array_equal(out, 1.5 * prod - 2.0 * C)


@pytest.mark.parametrize("side", [0, 1])
@pytest.mark.parametrize("uplo", [0, 1])
@pytest.mark.parametrize("ta", [0, 1])
@pytest.mark.parametrize("diag", [0, 1])
def test_dtrmm_integer_exact(side, uplo, ta, diag):
    """The other triangle holds NaN and a unit diagonal holds NaN too (neither may
    be read); the result equals the exact integer product with the triangle."""
    rng = np.random.default_rng(60 + 8 * side + 4 * uplo + 2 * ta + diag)
    m, n = 19, 13
    k = m if side == 0 else n
    A = rng.integers(-8, 9, size=(k, k)).astype(np.float64)
    T = np.tril(A) if uplo == 0 else np.triu(A)
    if diag:
        np.fill_diagonal(T, 1.0)
    Anan = A.copy()
    Anan[np.triu_indices(k, 1) if uplo == 0 else np.tril_indices(k, -1)] = np.nan
    if diag:
        np.fill_diagonal(Anan, np.nan)
    B = rng.integers(-8, 9, size=(m, n)).astype(np.float64)
    out = oracle.dtrmm(np.asfortranarray(Anan), B, 2.0, side, uplo, ta, diag)
    op = (T.T if ta else T).astype(np.int64)
    prod = (op @ B.astype(np.int64) if side == 0 else B.astype(np.int64) @ op).astype(np.float64)
    np.testing.assert_array_equal(out, 2.0 * prod)


@pytest.mark.parametrize("side", [0, 1])
@pytest.mark.parametrize("uplo", [0, 1])
@pytest.mark.parametrize("ta", [0, 1])
@pytest.mark.parametrize("diag", [0, 1])
def test_dtrsm_recovers_integer_solution(side, uplo, ta, diag):
    """B = op(T) X (or X op(T)) for an integer X and a triangular T with small
    integers off the diagonal and a power-of-two (or unit) diagonal: every
    partial sum of the substitution is an exact integer multiple of a power of
    two, so the solve must return X bitwise.  The unread triangle holds NaN."""
    rng = np.random.default_rng(100 + 8 * side + 4 * uplo + 2 * ta + diag)
    m, n = 17, 11
    k = m if side == 0 else n
    A = rng.integers(-3, 4, size=(k, k)).astype(np.float64)
    np.fill_diagonal(A, rng.choice([-4.0, -2.0, -1.0, 1.0, 2.0, 4.0], size=k))
    T = np.tril(A) if uplo == 0 else np.triu(A)
    if diag:
        np.fill_diagonal(T, 1.0)
    op = T.T if ta else T
    X = rng.integers(-5, 6, size=(m, n)).astype(np.float64)
    B = op @ X if side == 0 else X @ op
    Anan = A.copy()
    Anan[np.triu_indices(k, 1) if uplo == 0 else np.tril_indices(k, -1)] = np.nan
    if diag:
        np.fill_diagonal(Anan, np.nan)
    out = oracle.dtrsm(np.asfortranarray(Anan), np.asfortranarray(2.0 * B), 0.5, side, uplo, ta, diag)
    np.testing.assert_array_equal(out, X)


# ---------------------------------------------------------------- Level-1/2
# The routines FT-BLAS protects by duplicated computation (§4): DSCAL, DNRM2,
# DGEMV, DTRSV.  Pinned by exact arithmetic, closed forms and library routines.

def test_dscal_exact_products_and_stride():
    """alpha = 3 times small integers and powers of two is exact; stride 2
    scales only the even positions; n <= 0 or incx <= 0 leave x unchanged;
    alpha = 0 multiplies (NaN stays NaN, as the BLAS definition has no
    special case)."""
    x = np.array([1.0, -2.0, 0.5, 2.0 ** -1000, 7.0, np.nan])
    np.testing.assert_array_equal(oracle.dscal(x, 6, 3.0), [3.0, -6.0, 1.5, 3 * 2.0 ** -1000, 21.0, np.nan])
    np.testing.assert_array_equal(oracle.dscal(x[:5], 3, -2.0, incx=2), [-2.0, -2.0, -1.0, 2.0 ** -1000, -14.0])
    np.testing.assert_array_equal(oracle.dscal(x, 0, 5.0), x)
    np.testing.assert_array_equal(oracle.dscal(x, 6, 5.0, incx=0), x)
    out = oracle.dscal(x, 6, 0.0)
    assert np.isnan(out[5]) and np.all(out[:5] == 0.0)


@pytest.mark.parametrize("v,expect", [
    ([3.0, 4.0], 5.0),
    ([1.0, 2.0, 2.0], 3.0),
    ([2.0, 3.0, 6.0], 7.0),
    ([0.0, 0.0], 0.0),
    ([-5.0], 5.0),
    ([1.0, 1.0, 1.0, 1.0], 2.0),
])
def test_dnrm2_closed_forms(v, expect):
    """Pythagorean triples and quadruples give exact norms; four equal entries
    give twice their magnitude."""
    assert oracle.dnrm2(np.array(v), len(v)) == expect


@pytest.mark.parametrize("e", [600, -600, -1070, 1000])
def test_dnrm2_no_overflow_or_underflow(e):
    """(3, 4, 12) 2^e has norm 13 2^e exactly, far outside the range where the
    plain sum of squares over- or underflows (2^-1070 is subnormal)."""
    s = 2.0 ** e
    assert oracle.dnrm2(np.array([3.0 * s, 4.0 * s, 12.0 * s]), 3) == 13.0 * s


def test_dnrm2_special_values_and_stride():
    assert math.isnan(oracle.dnrm2(np.array([1.0, np.nan, np.inf]), 3))
    assert oracle.dnrm2(np.array([1.0, -np.inf, 2.0]), 3) == math.inf
    assert oracle.dnrm2(np.array([3.0, 99.0, 4.0, 99.0]), 2, incx=2) == 5.0
    assert oracle.dnrm2(np.array([3.0, 4.0]), 0) == 0.0
    assert oracle.dnrm2(np.array([3.0, 4.0]), 2, incx=0) == 0.0


def test_dnrm2_matches_numpy_on_random_data():
    """Against numpy's norm (a library routine): both are within a few
    rounding units of the exact value for data this well scaled."""
    rng = np.random.default_rng(7)
    for n in (1, 17, 1000, 100003):
        x = rng.standard_normal(n)
        ref = float(np.linalg.norm(x))
        assert abs(oracle.dnrm2(x, n) - ref) <= 1e-14 * ref


def test_dgemv_integer_example_both_operations():
    """A = [[1, 2, 3], [4, 5, 6]]: A (1, 0, -1) = (-2, -2) and A^T (1, 1) =
    (5, 7, 9); alpha and beta apply as alpha op(A) x + beta y."""
    A = np.asfortranarray([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0]])
    np.testing.assert_array_equal(oracle.dgemv(A, [1.0, 0.0, -1.0], [0.0, 0.0]), [-2.0, -2.0])
    np.testing.assert_array_equal(oracle.dgemv(A, [1.0, 1.0], [0.0, 0.0, 0.0], ta=1), [5.0, 7.0, 9.0])
    np.testing.assert_array_equal(oracle.dgemv(A, [1.0, 0.0, -1.0], [10.0, 20.0], alpha=2.0, beta=0.5),
                                  [1.0, 6.0])
    # the transposed product is not the plain one: a swapped operand fails here
    np.testing.assert_array_equal(oracle.dgemv(A, [1.0, 2.0], [0.0, 0.0, 0.0], ta=1), [9.0, 12.0, 15.0])


def test_dgemv_negative_strides_and_beta_zero():
    """A negative increment walks the vector from the far end; beta = 0 does
    not read y (NaN there is ignored); alpha = 0 reads neither A nor x."""
    A = np.asfortranarray([[1.0, 2.0, 3.0], [4.0, 5.0, 6.0]])
    xb = [-1.0, 0.0, 1.0]  # with incx = -1 element 0 is the last entry: x = (1, 0, -1)
    np.testing.assert_array_equal(oracle.dgemv(A, xb, [np.nan, np.nan], incx=-1), [-2.0, -2.0])
    yb = [7.0, 99.0, 5.0]  # incy = -2: y = (5, 7), written back at the same places
    np.testing.assert_array_equal(oracle.dgemv(A, [1.0, 0.0, -1.0], yb, beta=1.0, incy=-2), [5.0, 99.0, 3.0])
    Anan = np.full((2, 3), np.nan, order="F")
    np.testing.assert_array_equal(oracle.dgemv(Anan, [np.nan] * 3, [2.0, 4.0], alpha=0.0, beta=3.0), [6.0, 12.0])


def test_dgemv_matches_numpy_within_bound():
    """Against numpy's matmul: |diff| <= 2 gamma_n (|A| |x|) elementwise (both
    sides are within gamma_n |A||x| of the exact product)."""
    rng = np.random.default_rng(3)
    for ta in (0, 1):
        A = np.asfortranarray(rng.standard_normal((37, 53)))
        lenx = 37 if ta else 53
        x = rng.standard_normal(lenx)
        out = oracle.dgemv(A, x, np.zeros(53 if ta else 37), ta=ta)
        op = A.T if ta else A
        g = lenx * 2.0 ** -53 / (1 - lenx * 2.0 ** -53)
        assert np.all(np.abs(out - op @ x) <= 2 * g * (np.abs(op) @ np.abs(x)))


@pytest.mark.parametrize("uplo", [0, 1])
@pytest.mark.parametrize("ta", [0, 1])
@pytest.mark.parametrize("diag", [0, 1])
@pytest.mark.parametrize("incx", [1, -2])
def test_dtrsv_recovers_integer_solution(uplo, ta, diag, incx):
    """b = op(T) x for an integer x and a triangular T with small integers off
    the diagonal and a power-of-two (or unit) diagonal: every partial sum is
    exact, so the solve returns x bitwise; the unread triangle (and a unit
    diagonal) hold NaN."""
    rng = np.random.default_rng(200 + 8 * uplo + 4 * ta + 2 * diag + (incx < 0))
    n = 23
    A = rng.integers(-3, 4, size=(n, n)).astype(np.float64)
    np.fill_diagonal(A, rng.choice([-4.0, -2.0, -1.0, 1.0, 2.0, 4.0], size=n))
    T = np.tril(A) if uplo == 0 else np.triu(A)
    if diag:
        np.fill_diagonal(T, 1.0)
    op = T.T if ta else T
    x = rng.integers(-5, 6, size=n).astype(np.float64)
    b = op @ x
    Anan = A.copy()
    Anan[np.triu_indices(n, 1) if uplo == 0 else np.tril_indices(n, -1)] = np.nan
    if diag:
        np.fill_diagonal(Anan, np.nan)
    buf = np.full(1 + (n - 1) * abs(incx), 123.0)
    pos = np.arange(n) * abs(incx)
    if incx < 0:
        pos = pos[::-1]
    buf[pos] = b
    out = oracle.dtrsv(np.asfortranarray(Anan), buf, uplo, ta, diag, incx)
    np.testing.assert_array_equal(out[pos], x)
    mask = np.ones(buf.size, bool)
    mask[pos] = False
    assert np.all(out[mask] == 123.0)
