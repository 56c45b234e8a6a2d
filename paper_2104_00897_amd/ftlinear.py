"""Fault-tolerant linear layer: Y = X W^T with every product a protected GEMM.

Row-major torch tensors map onto the column-major C ABI without copies:
a row-major (r x c) tensor is a column-major (c x r) matrix, so
    forward   Y^T  = W^T X^T     -> ftg (T, N), m = out, n = tokens, k = in
    input     dX^T = W^T dY^T    -> ftg (N, N), m = in,  n = tokens, k = out
    weight    dW^T = X^T dY      -> ftg (N, T), m = in,  n = out,    k = tokens
(the three GEMMs of a linear layer's training step).  bfloat16 operands run
through ftg_gemm_ex (FP32 accumulation, checksums and verification), and the
FP32 results are rounded to bfloat16 after verification; float64 operands run
through ftg_dgemm.  Every step runs in the HIP library; there is no fallback.
"""
from __future__ import annotations

import torch

from . import ftgemm


def _check(t: torch.Tensor, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (row-major)")


def _gemm(handle, ta, tb, m, n, k, A, lda, B, ldb, C, ldc, cfg):
    """C (column-major m x n, leading dimension ldc) := op(A) op(B)."""
    stream = ftgemm.current_stream_ptr()
    if A.dtype == torch.float64:
        handle.dgemm(ta, tb, m, n, k, 1.0, ftgemm.ptr(A), lda, ftgemm.ptr(B), ldb, 0.0,
                     ftgemm.ptr(C), ldc, stream, cfg)
    else:
        handle.gemm_ex(ta, tb, m, n, k, ftgemm.BF16, ftgemm.F32, None, None, 1.0, ftgemm.ptr(A),
                       lda, ftgemm.ptr(B), ldb, 0.0, ftgemm.ptr(C), ldc, stream, cfg)


def _out(rows_major: int, cols_major: int, like: torch.Tensor):
    """Result buffer of a row-major (rows x cols) result: float64 or FP32 staging."""
    dt = torch.float64 if like.dtype == torch.float64 else torch.float32
    return torch.empty((rows_major, cols_major), dtype=dt, device=like.device)


def _finish(C: torch.Tensor, like: torch.Tensor):
    # bfloat16 outputs are rounded after verification (outside the protected sphere)
    return C if like.dtype == torch.float64 else C.to(torch.bfloat16)


class FTLinearFunction(torch.autograd.Function):
    """Y = X W^T; X (tokens x in), W (out x in), both row-major, bfloat16 or float64."""

    @staticmethod
    def forward(ctx, X, W, handle, cfg_fwd, cfg_bwd):
        _check(X, "X")
        _check(W, "W")
        if X.dtype != W.dtype or X.dtype not in (torch.bfloat16, torch.float64):
            raise ValueError("X and W must both be bfloat16 or both float64")
        T, din = X.shape
        dout = W.shape[0]
        if W.shape[1] != din:
            raise ValueError("W must be (out x in) with in = X.shape[1]")
        Y = _out(T, dout, X)
        # Y^T (out x T) = op(A) op(B), A = W as column-major (in x out) transposed, B = X^T
        _gemm(handle, ftgemm.OP_T, ftgemm.OP_N, dout, T, din, W, din, X, din, Y, dout, cfg_fwd)
        ctx.save_for_backward(X, W)
        ctx.handle, ctx.cfg_bwd = handle, cfg_bwd
        return _finish(Y, X)

    @staticmethod
    def backward(ctx, dY):
        X, W = ctx.saved_tensors
        h, cfg = ctx.handle, ctx.cfg_bwd
        dY = dY.to(X.dtype).contiguous()
        T, din = X.shape
        dout = W.shape[0]
        dX = dW = None
        if ctx.needs_input_grad[0]:
            dX = _out(T, din, X)
            # dX^T (in x T) = W^T (in x out) dY^T (out x T)
            _gemm(h, ftgemm.OP_N, ftgemm.OP_N, din, T, dout, W, din, dY, dout, dX, din, cfg)
            dX = _finish(dX, X)
        if ctx.needs_input_grad[1]:
            dW = _out(dout, din, X)
            # dW^T (in x out) = X^T (in x T) dY (T x out)
            _gemm(h, ftgemm.OP_N, ftgemm.OP_T, din, dout, T, X, din, dY, dout, dW, din, cfg)
            dW = _finish(dW, X)
        return dX, dW, None, None, None


def ft_linear(X, W, handle, cfg_fwd=None, cfg_bwd=None):
    """Fault-tolerant Y = X W^T (see FTLinearFunction)."""
    return FTLinearFunction.apply(X, W, handle, cfg_fwd, cfg_bwd)


class FTLinear(torch.nn.Module):
    """Bias-free linear layer whose forward and backward products are protected."""

    def __init__(self, in_features, out_features, handle, dtype=torch.bfloat16, device="cuda",
                 cfg_fwd=None, cfg_bwd=None, init_std=0.02, generator=None):
        super().__init__()
        w = torch.randn(out_features, in_features, generator=generator, dtype=torch.float32,
                        device="cpu") * init_std
        self.weight = torch.nn.Parameter(w.to(dtype).to(device))
        self.handle, self.cfg_fwd, self.cfg_bwd = handle, cfg_fwd, cfg_bwd

    def forward(self, X):
        return ft_linear(X, self.weight, self.handle, self.cfg_fwd, self.cfg_bwd)
