"""GPU parity of FT-DTRSM (blocked triangular solve: protected GEMM updates and
checksum-verified diagonal-block solves, §3.3.3), through the C ABI, against
the CPU oracle's substitution.

Operands are well conditioned (diagonal in [1, 2], off-diagonal entries of
size 0.5/k), so the blocked and the substitution orders agree closely:
  * the backward error of the result, |op(A) X - alpha B| componentwise
    against the rounding bound (checked in binary64 on the host);
  * the forward error against the oracle, normwise;
  * integer data with a unit diagonal: bitwise equal to the oracle;
  * injected faults (in the updates and in the diagonal solves) corrected."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2104_00897_amd import ftgemm
    assert torch.cuda.is_available()
    h = ftgemm.Handle(capacity=8192)
    yield ftgemm, h, torch
    torch.cuda.synchronize()
    h.close()


def well_conditioned(rng, k, uplo, diag):
    """Triangular A (stored full, the unread triangle and a unit diagonal set to NaN)
    and its op-ready dense triangle."""
    A = rng.uniform(-1, 1, (k, k)) * (0.5 / k)
    np.fill_diagonal(A, rng.uniform(1, 2, k) * rng.choice([-1.0, 1.0], k))
    T = np.tril(A) if uplo == 0 else np.triu(A)
    if diag:
        np.fill_diagonal(T, 1.0)
    Ah = A.copy()
    Ah[np.triu_indices(k, 1) if uplo == 0 else np.tril_indices(k, -1)] = np.nan
    if diag:
        np.fill_diagonal(Ah, np.nan)
    return np.asfortranarray(Ah), T


def run(env, Ah, B, alpha, side, uplo, ta, diag, cfg=None):
    ftgemm, h, torch = env
    dA, dB = ftgemm.to_device(Ah), ftgemm.to_device(B)
    h.reset()
    ftgemm.dtrsm_f64(h, dA, dB, alpha, side, uplo, ta, diag, cfg)
    torch.cuda.synchronize()
    return ftgemm.to_host(dB), h.read()


def check_solution(X, T, B, alpha, side, ta, ref):
    op = T.T if ta else T
    k = op.shape[0]
    R = (op @ X if side == 0 else X @ op) - alpha * B
    M = (np.abs(op) @ np.abs(X) if side == 0 else np.abs(X) @ np.abs(op)) + abs(alpha) * np.abs(B)
    gam = 4.0 * (2 * k + 8) * U
    assert np.all(np.abs(R) <= gam * M), float(np.max(np.abs(R) / M))
    assert np.linalg.norm(X - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("side", [0, 1])
@pytest.mark.parametrize("uplo", [0, 1])
@pytest.mark.parametrize("ta", [0, 1])
@pytest.mark.parametrize("diag", [0, 1])
def test_dtrsm_matches_oracle(env, side, uplo, ta, diag):
    """Sizes span two outer blocks of 1024 and several 256 diagonal blocks, with
    ragged last blocks."""
    ftgemm = env[0]
    rng = np.random.default_rng(120 + 8 * side + 4 * uplo + 2 * ta + diag)
    m, n = (1300, 190) if side == 0 else (190, 1300)
    k = m if side == 0 else n
    Ah, T = well_conditioned(rng, k, uplo, diag)
    B = np.asfortranarray(rng.uniform(-1, 1, (m, n)))
    ref = oracle.dtrsm(Ah, B, 1.5, side, uplo, ta, diag)
    X, rep = run(env, Ah, B, 1.5, side, uplo, ta, diag)
    assert rep.detected == 0 and 0.0 < rep.max_pass_ratio < 0.5
    check_solution(X, T, B, 1.5, side, ta, ref)
    # unprotected run of the same blocking
    Xu, _ = run(env, Ah, B, 1.5, side, uplo, ta, diag, ftgemm.make_config(abft=False))
    check_solution(Xu, T, B, 1.5, side, ta, ref)


@pytest.mark.parametrize("side", [0, 1])
def test_dtrsm_faults_corrected(env, side):
    """Exponent flips in every protected step (the updates' accumulators and the
    diagonal solves' unknowns) are all corrected; the result is unchanged."""
    ftgemm = env[0]
    rng = np.random.default_rng(130 + side)
    m, n = (1100, 300) if side == 0 else (300, 1100)
    k = m if side == 0 else n
    Ah, T = well_conditioned(rng, k, 0, 0)
    B = np.asfortranarray(rng.uniform(-1, 1, (m, n)))
    ref = oracle.dtrsm(Ah, B, -2.0, side, 0, 0, 0)
    cfg = ftgemm.make_config(seed=11, n_faults=2, bit_lo=56, bit_hi=62)
    X, rep = run(env, Ah, B, -2.0, side, 0, 0, 0, cfg)
    assert rep.injected >= 8 and rep.uncorrectable == 0
    assert rep.corrected_subtract + rep.corrected_recompute == rep.injected
    solves = [r for r in rep.records if r["row"] == -1]
    assert solves and all(r["kind"] == ftgemm.KIND_RECOMPUTE for r in solves)
    check_solution(X, T, B, -2.0, side, 0, ref)


def test_dtrsm_integer_bitwise_alpha_zero_and_errors(env):
    ftgemm, h, torch = env
    rng = np.random.default_rng(140)
    m, n = 600, 70
    A = rng.integers(-1, 2, size=(m, m)).astype(np.float64)
    T = np.tril(A, -1) + np.eye(m)
    X = rng.integers(-3, 4, size=(m, n)).astype(np.float64)
    B = np.asfortranarray(T @ X)
    assert np.abs(B).max() < 2 ** 40
    Ah = np.asfortranarray(np.tril(A, -1) + np.triu(np.full((m, m), np.nan)))
    out, rep = run(env, Ah, B, 1.0, 0, 0, 0, 1)
    np.testing.assert_array_equal(out, oracle.dtrsm(Ah, B, 1.0, 0, 0, 0, 1))
    np.testing.assert_array_equal(out, X)
    out, _ = run(env, np.full((m, m), np.nan, order="F"), B, 0.0, 0, 0, 0, 0)
    np.testing.assert_array_equal(out, np.zeros((m, n)))
    d = torch.zeros(64, dtype=torch.float64, device="cuda")
    p = ftgemm.ptr(d)
    for args, info in [((2, 0, 0, 0, 4, 4), 1), ((0, 3, 0, 0, 4, 4), 2), ((0, 0, 2, 0, 4, 4), 3),
                       ((0, 0, 0, 2, 4, 4), 4), ((0, 0, 0, 0, -1, 4), 5), ((0, 0, 0, 0, 4, -1), 6)]:
        with pytest.raises(ftgemm.FtgError) as e:
            h.dtrsm(*args, 1.0, p, 4, p, 4)
        assert e.value.info == info
