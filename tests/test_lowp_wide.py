"""GPU parity of the wide low-precision tile (configuration 2: 256 x 256 outputs per
workgroup, eight waves of 128 x 64; bf16, and fp8 on the full-rate f8f6f4 MFMA,
plain and protected) against the CPU oracle, through the C ABI.

Same bars as the 128 x 128 kernel: integer-exact inputs give the oracle's result
bitwise (FP32 accumulation is exact there), random inputs stay within the
rigorous FP32 accumulation bound 2 (k + 2) u32 M.  Shapes cover several wide
tiles with ragged edges in m and n, a C whose leading dimension rules out
16-byte stores, every transpose pair (packed to k-contiguous operands first) and
a k that is not a multiple of the k-block (the 128 x 128 kernel then runs)."""
import numpy as np
import pytest

from tests.test_parity_lowp import Run, assert_close32, check_flips, env, plan_for  # noqa: F401

pytestmark = pytest.mark.gpu

WIDE = 2


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("m,n,k", [(520, 300, 192), (301, 530, 96), (257, 256, 32)])
def test_wide_integer_exact_bitwise(env, ta, tb, m, n, k):
    ftgemm = env[0]
    r = Run(env, "bf16", m, n, k, ta, tb, seed=31, integer=True)
    for alpha, beta in [(1.0, 0.0), (-2.0, 0.5)]:
        out, _ = r.gpu(alpha, beta, ftgemm.make_config(abft=False, tile=WIDE), nan_c=(beta == 0.0))
        np.testing.assert_array_equal(out, r.oracle(alpha, beta))
        ref, _ = r.gpu(alpha, beta, ftgemm.make_config(abft=False, tile=1), nan_c=(beta == 0.0))
        np.testing.assert_array_equal(out, ref)


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0)])
def test_wide_random_within_fp32_bound(env, ta, tb):
    ftgemm = env[0]
    r = Run(env, "bf16", 600, 650, 1024, ta, tb, seed=32)
    for alpha, beta in [(1.0, 0.0), (1.5, 0.5)]:
        out, _ = r.gpu(alpha, beta, ftgemm.make_config(abft=False, tile=WIDE))
        assert_close32(out, r.oracle(alpha, beta), r.magnitude(alpha, beta), r.k)


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("m,n,k", [(520, 300, 192), (257, 513, 64), (300, 290, 320)])
def test_wide_fp8_integer_exact_bitwise(env, ta, tb, m, n, k):
    """fp8 on the full-rate 32x32x64 f8f6f4 MFMA (k a multiple of its 64-step
    k-block): integer-valued e4m3 inputs give the oracle's result bitwise, equal
    to the 128 x 128 kernel's."""
    ftgemm = env[0]
    r = Run(env, "fp8", m, n, k, ta, tb, seed=38, integer=True)
    for alpha, beta in [(1.0, 0.0), (-2.0, 0.5)]:
        out, _ = r.gpu(alpha, beta, ftgemm.make_config(abft=False, tile=WIDE), nan_c=(beta == 0.0))
        np.testing.assert_array_equal(out, r.oracle(alpha, beta))
        ref, _ = r.gpu(alpha, beta, ftgemm.make_config(abft=False, tile=1), nan_c=(beta == 0.0))
        np.testing.assert_array_equal(out, ref)


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0)])
def test_wide_fp8_random_within_fp32_bound(env, ta, tb):
    ftgemm = env[0]
    r = Run(env, "fp8", 600, 650, 1024, ta, tb, seed=39)
    for alpha, beta in [(1.0, 0.0), (1.5, 0.5)]:
        out, _ = r.gpu(alpha, beta, ftgemm.make_config(abft=False, tile=WIDE))
        assert_close32(out, r.oracle(alpha, beta), r.magnitude(alpha, beta), r.k)


def test_wide_k_tail_falls_back(env):
    """k = 197 is no multiple of the 32-step k-block: the call takes the 128 x 128
    kernel and still matches the oracle bitwise on integer inputs."""
    ftgemm = env[0]
    r = Run(env, "bf16", 300, 280, 197, 1, 0, seed=33, integer=True)
    out, _ = r.gpu(1.0, 1.0, ftgemm.make_config(abft=False, tile=WIDE))
    np.testing.assert_array_equal(out, r.oracle(1.0, 1.0))


# ---- protected: the checksums folded into the wide product (2 x 2 checksum
# tiles of 128 x 128 per workgroup, the same slots and thresholds as tile 1)

@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_wide_protected_integer_exact(env, ta, tb):
    ftgemm = env[0]
    r = Run(env, "bf16", 520, 300, 192, ta, tb, seed=34, integer=True)
    for alpha, beta in [(1.0, 0.0), (1.0, 1.0), (-2.0, 0.5)]:
        out, rep = r.gpu(alpha, beta, ftgemm.make_config(tile=WIDE), nan_c=(beta == 0.0))
        np.testing.assert_array_equal(out, r.oracle(alpha, beta))
        assert rep.detected == 0, rep.records[:3]


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0)])
def test_wide_protected_random_no_false_flags(env, ta, tb):
    ftgemm = env[0]
    r = Run(env, "bf16", 600, 650, 1024, ta, tb, seed=35)
    for alpha, beta in [(1.0, 0.0), (1.5, 0.5)]:
        out, rep = r.gpu(alpha, beta, ftgemm.make_config(tile=WIDE))
        assert_close32(out, r.oracle(alpha, beta), r.magnitude(alpha, beta), r.k)
        assert rep.detected == 0, rep.records[:3]


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0)])
def test_wide_flips_located_and_corrected(env, ta, tb):
    ftgemm = env[0]
    r = Run(env, "bf16", 530, 400, 704, ta, tb, seed=36)
    F = 12
    for alpha, beta in [(1.0, 0.0), (1.5, 0.5)]:
        cfg = ftgemm.make_config(seed=31, n_faults=F, bit_lo=24, bit_hi=30, tile=WIDE)
        out, rep = r.gpu(alpha, beta, cfg)
        plan = plan_for(r, 31, F, 24, 30)
        assert rep.injected == F and rep.uncorrectable == 0
        assert check_flips(r, alpha, beta, out, rep, plan) >= F // 2


def test_wide_checksum_target_and_two_in_slot(env):
    ftgemm = env[0]
    r = Run(env, "bf16", 256, 384, 320, 0, 0, seed=37)
    cfg = ftgemm.make_config(seed=3, n_faults=4, bit_lo=25, bit_hi=30, target=ftgemm.TARGET_CHECKSUM, tile=WIDE)
    out, rep = r.gpu(1.0, 1.0, cfg)
    assert rep.injected == 4 and rep.checksum_only == 4
    assert all(g["kind"] == ftgemm.KIND_CHECKSUM_ONLY and g["col"] == -1 for g in rep.records)
    assert_close32(out, r.oracle(1.0, 1.0), r.magnitude(1.0, 1.0), r.k)
    cfg = ftgemm.make_config(seed=5, n_faults=2, bit_lo=26, bit_hi=30, target=ftgemm.TARGET_TWO_IN_SLOT,
                             tile=WIDE)
    out, rep = r.gpu(1.0, 0.0, cfg)
    assert rep.injected == 4 and rep.uncorrectable == 2 and rep.status == ftgemm.ERR_UNCORRECTED


# ---- protected fp8: e4m3 checksum pieces (eight per panel sum, scales
# 2^(7 - 4 t)) multiplied on the fp8 MFMA

@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_wide_fp8_protected_integer_exact(env, ta, tb):
    ftgemm = env[0]
    r = Run(env, "fp8", 520, 300, 192, ta, tb, seed=40, integer=True)
    for alpha, beta in [(1.0, 0.0), (1.0, 1.0), (-2.0, 0.5)]:
        out, rep = r.gpu(alpha, beta, ftgemm.make_config(tile=WIDE), nan_c=(beta == 0.0))
        np.testing.assert_array_equal(out, r.oracle(alpha, beta))
        assert rep.detected == 0, rep.records[:3]


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0)])
def test_wide_fp8_protected_random_no_false_flags(env, ta, tb):
    ftgemm = env[0]
    r = Run(env, "fp8", 600, 650, 1024, ta, tb, seed=41)
    for alpha, beta in [(1.0, 0.0), (1.5, 0.5)]:
        out, rep = r.gpu(alpha, beta, ftgemm.make_config(tile=WIDE))
        assert_close32(out, r.oracle(alpha, beta), r.magnitude(alpha, beta), r.k)
        assert rep.detected == 0, rep.records[:3]


@pytest.mark.parametrize("ta,tb", [(0, 0), (1, 0)])
def test_wide_fp8_flips_located_and_corrected(env, ta, tb):
    ftgemm = env[0]
    r = Run(env, "fp8", 530, 400, 704, ta, tb, seed=42)
    F = 12
    for alpha, beta in [(1.0, 0.0), (1.5, 0.5)]:
        cfg = ftgemm.make_config(seed=31, n_faults=F, bit_lo=24, bit_hi=30, tile=WIDE)
        out, rep = r.gpu(alpha, beta, cfg)
        plan = plan_for(r, 31, F, 24, 30)
        assert rep.injected == F and rep.uncorrectable == 0
        assert check_flips(r, alpha, beta, out, rep, plan) >= F // 2


def test_wide_fp8_checksum_target_and_two_in_slot(env):
    ftgemm = env[0]
    r = Run(env, "fp8", 256, 384, 320, 0, 0, seed=43)
    cfg = ftgemm.make_config(seed=3, n_faults=4, bit_lo=25, bit_hi=30, target=ftgemm.TARGET_CHECKSUM, tile=WIDE)
    out, rep = r.gpu(1.0, 1.0, cfg)
    assert rep.injected == 4 and rep.checksum_only == 4
    assert_close32(out, r.oracle(1.0, 1.0), r.magnitude(1.0, 1.0), r.k)
    cfg = ftgemm.make_config(seed=5, n_faults=2, bit_lo=26, bit_hi=30, target=ftgemm.TARGET_TWO_IN_SLOT,
                             tile=WIDE)
    out, rep = r.gpu(1.0, 0.0, cfg)
    assert rep.injected == 4 and rep.uncorrectable == 2 and rep.status == ftgemm.ERR_UNCORRECTED


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
def test_wide_protected_edges(env, kind):
    """Protected wide calls on a C whose leading dimension rules out 16-byte
    stores (m = 301), with beta != 0 (the tile is stored by a second pass after
    the checks) and with a NaN-filled C at beta = 0 (C is not read); a k that is
    no multiple of the k-block falls back to the 128 x 128 kernel."""
    ftgemm = env[0]
    r = Run(env, kind, 301, 530, 192, 0, 0, seed=44, integer=True)
    for alpha, beta in [(1.0, 0.0), (-2.0, 0.5)]:
        out, rep = r.gpu(alpha, beta, ftgemm.make_config(tile=WIDE), nan_c=(beta == 0.0))
        np.testing.assert_array_equal(out, r.oracle(alpha, beta))
        assert rep.detected == 0, rep.records[:3]
    r = Run(env, kind, 300, 280, 200, 1, 0, seed=45, integer=True)
    out, rep = r.gpu(1.0, 1.0, ftgemm.make_config(tile=WIDE))
    np.testing.assert_array_equal(out, r.oracle(1.0, 1.0))
    assert rep.detected == 0
