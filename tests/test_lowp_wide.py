"""GPU parity of the wide low-precision tile (configuration 2: 256 x 256 outputs per
workgroup, eight waves of 128 x 64) against the CPU oracle, through the C ABI.

Same bars as the 128 x 128 kernel: integer-exact inputs give the oracle's result
bitwise (FP32 accumulation is exact there), random inputs stay within the
rigorous FP32 accumulation bound 2 (k + 2) u32 M.  Shapes cover several wide
tiles with ragged edges in m and n, a C whose leading dimension rules out
16-byte stores, every transpose pair (packed to k-contiguous operands first) and
a k that is not a multiple of the k-block (the 128 x 128 kernel then runs)."""
import numpy as np
import pytest

from tests.test_parity_lowp import Run, assert_close32, env  # noqa: F401

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


def test_wide_k_tail_falls_back(env):
    """k = 197 is no multiple of the 32-step k-block: the call takes the 128 x 128
    kernel and still matches the oracle bitwise on integer inputs."""
    ftgemm = env[0]
    r = Run(env, "bf16", 300, 280, 197, 1, 0, seed=33, integer=True)
    out, _ = r.gpu(1.0, 1.0, ftgemm.make_config(abft=False, tile=WIDE))
    np.testing.assert_array_equal(out, r.oracle(1.0, 1.0))
