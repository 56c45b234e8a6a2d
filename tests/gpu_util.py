"""Helpers shared by the GPU parity tests (comparison bounds, device setup)."""
import numpy as np

U64 = 2.0 ** -53


def tol_f64(k):
    """Componentwise tolerance of the FP64 path: |C - C_oracle| <= tol * M with
    M = |alpha||op(A)||op(B)| + |beta||C_in| (the standard rounding bound 2 gamma_k,
    never below the 1e-12 target)."""
    return max(1e-12, 2.2 * k * U64)


def magnitude(A, B, C, alpha, beta, ta, tb):
    a = np.abs(A.T if ta else A)
    b = np.abs(B.T if tb else B)
    M = abs(alpha) * (a @ b)
    if beta != 0.0 and C is not None:
        M = M + abs(beta) * np.abs(C)
    return M


def assert_close_f64(C, ref, M, k, skip=None):
    err = np.abs(C - ref)
    bound = tol_f64(k) * M + 1e-300
    bad = err > bound
    if skip is not None:
        bad &= ~skip
    if bad.any():
        i, j = np.argwhere(bad)[0]
        raise AssertionError(f"{bad.sum()} elements out of bound; first ({i},{j}): "
                             f"gpu {C[i, j]!r} oracle {ref[i, j]!r} bound {bound[i, j]:.3e}")
    return float(np.max(err / (M + 1e-300)))
