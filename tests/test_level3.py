"""GPU parity of FT-DSYMM and FT-DTRMM (the Level-3 routines that run on the
protected product after packing, §6.2.3), through the C ABI, against the CPU
oracle's plain definitions.  The triangle that must not be read holds NaN on
the device; results must match the oracle within the componentwise rounding
bound (bitwise on integer inputs); injected faults must be corrected."""
import numpy as np
import pytest

import oracle
from paper_2104_00897_amd import inputs
from tests.gpu_util import assert_close_f64, tol_f64

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


def hide_triangle(A, uplo, diag=0):
    """A copy of A with the unread triangle (and a unit diagonal) set to NaN."""
    X = A.copy(order="F")
    k = A.shape[0]
    X[np.triu_indices(k, 1) if uplo == 0 else np.tril_indices(k, -1)] = np.nan
    if diag:
        np.fill_diagonal(X, np.nan)
    return X


def sym_full(A, uplo):
    L = np.tril(A) if uplo == 0 else np.triu(A)
    return L + (L.T - np.diag(np.diag(L)))


def tri_op(A, uplo, ta, diag):
    T = np.tril(A) if uplo == 0 else np.triu(A)
    if diag:
        np.fill_diagonal(T, 1.0)
    return T.T if ta else T


@pytest.mark.parametrize("side", [0, 1])
@pytest.mark.parametrize("uplo", [0, 1])
def test_dsymm_matches_oracle(env, side, uplo):
    ftgemm, h, torch = env
    m, n = 301, 286
    k = m if side == 0 else n
    rng = np.random.default_rng(70 + 2 * side + uplo)
    A = np.asfortranarray(rng.uniform(-1, 1, (k, k)))
    B = np.asfortranarray(rng.uniform(-1, 1, (m, n)))
    C = np.asfortranarray(rng.uniform(-1, 1, (m, n)))
    Ah = hide_triangle(A, uplo)
    ref = oracle.dsymm(Ah, B, C, 1.5, 0.5, side, uplo)
    full = np.abs(sym_full(A, uplo))
    M = 1.5 * (full @ np.abs(B) if side == 0 else np.abs(B) @ full) + 0.5 * np.abs(C)
    for cfg in (None, ftgemm.make_config(seed=3, n_faults=6, bit_lo=52, bit_hi=62)):
        dA, dB, dC = ftgemm.to_device(Ah), ftgemm.to_device(B), ftgemm.to_device(C)
        h.reset()
        ftgemm.dsymm_f64(h, dA, dB, dC, 1.5, 0.5, side, uplo, cfg)
        torch.cuda.synchronize()
        rep = h.read()
        assert_close_f64(ftgemm.to_host(dC), ref, M, k)
        if cfg is not None:
            assert rep.injected == 6 and rep.corrected_subtract + rep.corrected_recompute == 6
        else:
            assert rep.detected == 0


def test_dsymm_integer_exact_and_errors(env):
    ftgemm, h, torch = env
    m, n = 130, 90
    A, B, C = inputs.integer_operands(m, n, m, seed=71)
    Ah = hide_triangle(A, 1)
    dA, dB, dC = ftgemm.to_device(Ah), ftgemm.to_device(B), ftgemm.to_device(C)
    ftgemm.dsymm_f64(h, dA, dB, dC, 2.0, -1.0, 0, 1)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ftgemm.to_host(dC), oracle.dsymm(Ah, B, C, 2.0, -1.0, 0, 1))
    p = ftgemm.ptr(dA)
    for args, info in [((2, 0, 4, 4), 1), ((0, 5, 4, 4), 2), ((0, 0, -1, 4), 3), ((0, 0, 4, -1), 4)]:
        with pytest.raises(ftgemm.FtgError) as e:
            h.dsymm(*args, 1.0, p, 4, p, 4, 0.0, p, 4)
        assert e.value.info == info
    with pytest.raises(ftgemm.FtgError) as e:
        h.dsymm(0, 0, 5, 4, 1.0, p, 4, p, 5, 0.0, p, 5)     # lda < m
    assert e.value.info == 7


@pytest.mark.parametrize("side", [0, 1])
@pytest.mark.parametrize("uplo", [0, 1])
@pytest.mark.parametrize("ta", [0, 1])
@pytest.mark.parametrize("diag", [0, 1])
def test_dtrmm_matches_oracle(env, side, uplo, ta, diag):
    ftgemm, h, torch = env
    # op(A) spans more than one 1024-wide block of the blocked product
    m, n = (1300, 211) if side == 0 else (211, 1300)
    k = m if side == 0 else n
    rng = np.random.default_rng(80 + 8 * side + 4 * uplo + 2 * ta + diag)
    A = np.asfortranarray(rng.uniform(-1, 1, (k, k)))
    B = np.asfortranarray(rng.uniform(-1, 1, (m, n)))
    Ah = hide_triangle(A, uplo, diag)
    ref = oracle.dtrmm(Ah, B, -1.5, side, uplo, ta, diag)
    op = np.abs(tri_op(A, uplo, ta, diag))
    M = 1.5 * (op @ np.abs(B) if side == 0 else np.abs(B) @ op)
    dA, dB = ftgemm.to_device(Ah), ftgemm.to_device(B)
    h.reset()
    cfg = ftgemm.make_config(seed=5, n_faults=3, bit_lo=52, bit_hi=62)
    ftgemm.dtrmm_f64(h, dA, dB, -1.5, side, uplo, ta, diag, cfg)
    torch.cuda.synchronize()
    rep = h.read()
    assert rep.uncorrectable == 0 and rep.injected >= 3
    # every flip far above any threshold here (tau <= 2 gamma(k + 136) 1.5 k 128 < 1e-7)
    # is corrected; a flip of an accumulator that is still exactly 0 (the zero part
    # of op(A) inside a block's k range) changes it by a denormal: masked
    fixed = {(r["row"], r["col"]) for r in rep.records if r["kind"] in (1, 2)}
    big = [g for g in rep.inject_log if not np.isfinite(g["new_val"]) or
           abs(g["new_val"] - g["old_val"]) * 1.5 > 1e-6]
    assert big and all((g["row"], g["col"]) in fixed for g in big)
    out = ftgemm.to_host(dB)
    err = np.abs(out - ref)
    assert np.all(err <= tol_f64(k) * M + 1e-300), float(np.max(err / (M + 1e-300)))


def test_dtrmm_integer_exact_alpha_zero_and_errors(env):
    ftgemm, h, torch = env
    m, n = 200, 150
    rng = np.random.default_rng(90)
    A = np.asfortranarray(rng.integers(-8, 9, (m, m)).astype(np.float64))
    B = np.asfortranarray(rng.integers(-8, 9, (m, n)).astype(np.float64))
    Ah = hide_triangle(A, 0, 1)
    dA, dB = ftgemm.to_device(Ah), ftgemm.to_device(B)
    ftgemm.dtrmm_f64(h, dA, dB, 2.0, 0, 0, 1, 1)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ftgemm.to_host(dB), oracle.dtrmm(Ah, B, 2.0, 0, 0, 1, 1))
    # alpha = 0: B := 0 without reading A (all NaN)
    dN = ftgemm.to_device(np.full((m, m), np.nan, order="F"))
    ftgemm.dtrmm_f64(h, dN, dB, 0.0, 0, 0, 0, 0)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ftgemm.to_host(dB), np.zeros((m, n)))
    p = ftgemm.ptr(dA)
    for args, info in [((2, 0, 0, 0, 4, 4), 1), ((0, 3, 0, 0, 4, 4), 2), ((0, 0, 2, 0, 4, 4), 3),
                       ((0, 0, 0, 2, 4, 4), 4), ((0, 0, 0, 0, -1, 4), 5), ((0, 0, 0, 0, 4, -1), 6)]:
        with pytest.raises(ftgemm.FtgError) as e:
            h.dtrmm(*args, 1.0, p, 4, p, 4)
        assert e.value.info == info
