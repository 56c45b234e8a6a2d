"""The differentiation pattern: FTLinear (Y = X W^T) whose forward and both backward
products are protected GEMMs through the C ABI.

Pins: L = <G, X W^T> is bilinear, so a central difference in X or W with any
step is exact up to rounding (no truncation term) and must equal the analytic
gradients G W and G^T X (float64, 64 x 64 x 64).  bfloat16 layers: every output
against the oracle's binary64 product of the same bfloat16 values, within the
FP32 accumulation bound plus the final bfloat16 rounding; faults injected into
the backward products are corrected."""
import numpy as np
import pytest

import oracle
from paper_2104_00897_amd import inputs
from tests.gpu_util import acc32_fault_taus, check_flip_values

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
UBF = 2.0 ** -8


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2104_00897_amd import ftgemm, ftlinear
    assert torch.cuda.is_available()
    h = ftgemm.Handle(capacity=8192)
    yield ftgemm, ftlinear, h, torch
    torch.cuda.synchronize()
    h.close()


def bf16_tensor(torch, rng, rows, cols, std):
    """Row-major bfloat16 device tensor and its exact values (float64, rows x cols)."""
    x = (rng.standard_normal((rows, cols)) * std).astype(np.float32)
    bits = inputs.to_bf16_bits(x)
    t = torch.from_numpy(bits.view(np.int16).copy()).view(torch.bfloat16).cuda()
    return t, inputs.bf16_bits_to_f64(bits)


def test_fd_gradients_float64(env):
    ftgemm, ftlinear, h, torch = env
    rng = np.random.default_rng(0)
    T = din = dout = 64
    Xn = rng.standard_normal((T, din)); Wn = rng.standard_normal((dout, din)); Gn = rng.standard_normal((T, dout))
    X = torch.tensor(Xn, device="cuda", requires_grad=True)
    W = torch.tensor(Wn, device="cuda", requires_grad=True)
    G = torch.tensor(Gn, device="cuda")
    Y = ftlinear.ft_linear(X, W, h)
    Y.backward(G)
    dX, dW = X.grad.cpu().numpy(), W.grad.cpu().numpy()

    def loss(Xh, Wh):
        with torch.no_grad():
            y = ftlinear.ft_linear(torch.tensor(Xh, device="cuda"), torch.tensor(Wh, device="cuda"), h)
        return float((y.cpu().numpy() * Gn).sum())

    scale = np.abs(Gn).sum() * np.abs(Wn).max() * np.abs(Xn).max() * din
    for _ in range(8):
        a, b = rng.integers(0, T), rng.integers(0, din)
        E = np.zeros_like(Xn); E[a, b] = 1.0
        fd = (loss(Xn + E, Wn) - loss(Xn - E, Wn)) / 2.0
        assert abs(fd - dX[a, b]) <= 1e-13 * scale, (a, b, fd, dX[a, b])
        c, d = rng.integers(0, dout), rng.integers(0, din)
        E = np.zeros_like(Wn); E[c, d] = 1.0
        fd = (loss(Xn, Wn + E) - loss(Xn, Wn - E)) / 2.0
        assert abs(fd - dW[c, d]) <= 1e-13 * scale, (c, d, fd, dW[c, d])
    # and the full gradients against the closed forms G W, G^T X
    np.testing.assert_allclose(dX, Gn @ Wn, rtol=0, atol=1e-12 * np.abs(Gn).sum(1).max() * np.abs(Wn).max())
    np.testing.assert_allclose(dW, Gn.T @ Xn, rtol=0, atol=1e-12 * np.abs(Gn).sum(0).max() * np.abs(Xn).max())


def close_bf16(got, ref, M, k):
    """FP32 accumulation bound plus the final rounding to bfloat16."""
    bound = 2.0 * (k + 2) * U32 * M + UBF * np.abs(ref) + 1e-30
    bad = np.abs(got - ref) > bound
    assert not bad.any(), (np.argwhere(bad)[:3], bad.sum())


def test_bf16_layer_with_backward_faults(env):
    ftgemm, ftlinear, h, torch = env
    rng = np.random.default_rng(1)
    T, din, dout = 300, 200, 150
    X, Xv = bf16_tensor(torch, rng, T, din, 1.0)
    W, Wv = bf16_tensor(torch, rng, dout, din, 1.0)
    G, Gv = bf16_tensor(torch, rng, T, dout, 1.0)
    X.requires_grad_(True); W.requires_grad_(True)
    bwd = ftgemm.make_config(seed=12, n_faults=3, bit_lo=26, bit_hi=30)
    h.reset()
    Y = ftlinear.ft_linear(X, W, h, None, bwd)
    Y.backward(G)
    torch.cuda.synchronize()
    rep = h.read()
    assert rep.injected == 6 and rep.uncorrectable == 0
    assert rep.corrected_subtract + rep.corrected_recompute == rep.detected == 6
    f64 = lambda t: t.detach().float().cpu().numpy().astype(np.float64)
    close_bf16(f64(Y), oracle.gemm(Xv, Wv, tb=1), np.abs(Xv) @ np.abs(Wv).T, din)
    close_bf16(f64(X.grad), oracle.gemm(Gv, Wv), np.abs(Gv) @ np.abs(Wv), dout)
    close_bf16(f64(W.grad), oracle.gemm(Gv, Xv, ta=1), np.abs(Gv).T @ np.abs(Xv), T)


def test_cfg4_full_size_sampled(env):
    """Tokens 8192, in 4096, out 4096; X, W ~ N(0, 0.02), dY ~ N(0, 1) in bfloat16;
    16 flips (bits 24..30) in each backward GEMM; sampled outputs against the oracle."""
    ftgemm, ftlinear, h, torch = env
    rng = np.random.default_rng(0)
    T, din, dout = 8192, 4096, 4096
    X, Xv = bf16_tensor(torch, rng, T, din, 0.02)
    W, Wv = bf16_tensor(torch, rng, dout, din, 0.02)
    G, Gv = bf16_tensor(torch, rng, T, dout, 1.0)
    X.requires_grad_(True); W.requires_grad_(True)
    bwd = ftgemm.make_config(seed=4, n_faults=16, bit_lo=24, bit_hi=30)
    h.reset()
    Y = ftlinear.ft_linear(X, W, h, None, bwd)
    Y.backward(G)
    torch.cuda.synchronize()
    rep = h.read()
    assert rep.injected == 32 and rep.uncorrectable == 0 and len(rep.inject_log) == 32
    check_flip_values(rep.inject_log, acc32=True)
    # A10 on both backward GEMMs (the kernels run in order, so the first 16 log
    # entries belong to dX^T = W^T dY^T, the last 16 to dW^T = X^T dY), each as
    # column-major op(A) (m x k) and op(B) (k x n) of exact values
    lam = ftgemm.default_lambda()
    taus = acc32_fault_taus(Wv.T, Gv.T, 1.0, rep.inject_log[:16], lam) + \
        acc32_fault_taus(Xv.T, Gv, 1.0, rep.inject_log[16:], lam)
    fixed = {(g["row"], g["col"]) for g in rep.records if g["kind"] in (1, 2)}
    big = 0
    for q, (g, tau) in enumerate(zip(rep.inject_log, taus)):
        d = abs(g["new_val"] - g["old_val"])
        if not np.isfinite(d) or d >= 4 * tau:
            big += 1
            assert (g["row"], g["col"]) in fixed, (q, g, tau)
    assert big >= 8
    s = 64
    r1, c1 = rng.integers(0, T, s), rng.integers(0, dout, s)
    ref = oracle.gemm_entries(Xv, Wv, None, r1, c1, tb=1)
    got = Y.detach().float()[torch.tensor(r1, device="cuda"), torch.tensor(c1, device="cuda")].double().cpu().numpy()
    M = np.array([np.dot(np.abs(Xv[i]), np.abs(Wv[j])) for i, j in zip(r1, c1)])
    assert np.all(np.abs(got - ref) <= 2 * (din + 2) * U32 * M + UBF * np.abs(ref))
    r2, c2 = rng.integers(0, T, s), rng.integers(0, din, s)
    ref = oracle.gemm_entries(Gv, Wv, None, r2, c2)
    got = X.grad.float()[torch.tensor(r2, device="cuda"), torch.tensor(c2, device="cuda")].double().cpu().numpy()
    M = np.array([np.dot(np.abs(Gv[i]), np.abs(Wv[:, j])) for i, j in zip(r2, c2)])
    assert np.all(np.abs(got - ref) <= 2 * (dout + 2) * U32 * M + UBF * np.abs(ref))
    r3, c3 = rng.integers(0, dout, s), rng.integers(0, din, s)
    ref = oracle.gemm_entries(Gv, Xv, None, r3, c3, ta=1)
    got = W.grad.float()[torch.tensor(r3, device="cuda"), torch.tensor(c3, device="cuda")].double().cpu().numpy()
    M = np.array([np.dot(np.abs(Gv[:, i]), np.abs(Xv[:, j])) for i, j in zip(r3, c3)])
    assert np.all(np.abs(got - ref) <= 2 * (T + 2) * U32 * M + UBF * np.abs(ref))
