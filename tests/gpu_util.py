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


def fp64_fault_taus(A, B, C, alpha, beta, ta, tb, log, bm, bn):
    """Detection threshold of each injected element (i, j) of an FP64 call: the
    larger of the thresholds of its tile row and tile column (a fault must
    clear both lines to be located), each 2 gamma(k + len + 8) M (1 + 2^-20)
    with the line's magnitude M computed here from the operands (the
    tile-local reading of the round-off threshold)."""
    import oracle
    a = np.abs(A.T if ta else A)
    b = np.abs(B.T if tb else B)
    m, k = a.shape
    n = b.shape[1]
    # per-tile panel sums: sum over the tile's columns of |b_pj| (k x tiles_n)
    # and over the tile's rows of |a_ip| (tiles_m x k)
    sb = np.add.reduceat(b, np.arange(0, n, bn), axis=1)
    sa = np.add.reduceat(a, np.arange(0, m, bm), axis=0)
    out = []
    for g in log:
        i, j = g["row"], g["col"]
        tm, tn = i // bm, j // bn
        R, Q = min(bm, m - tm * bm), min(bn, n - tn * bn)
        mr = abs(alpha) * float(a[i, :] @ sb[:, tn])
        mc = abs(alpha) * float(sa[tm, :] @ b[:, j])
        if beta != 0.0 and C is not None:
            mr += abs(beta) * float(np.abs(C[i, tn * bn:tn * bn + Q]).sum())
            mc += abs(beta) * float(np.abs(C[tm * bm:tm * bm + R, j]).sum())
        out.append(max(oracle.tau(k + Q + 8, mr), oracle.tau(k + R + 8, mc)))
    return out


def check_flip_values(log, acc32=False):
    """Every logged injection flipped exactly the logged bit of the logged old value
    (compared as bit patterns, so NaN results compare too)."""
    import oracle
    for g in log:
        if acc32:
            want = np.float32(oracle.flip32(np.float32(g["old_val"]), g["bit"]))
            got = np.float32(g["new_val"])
            assert want.view(np.uint32) == got.view(np.uint32), g
        else:
            want = np.float64(oracle.flip64(g["old_val"], g["bit"]))
            assert want.view(np.uint64) == np.float64(g["new_val"]).view(np.uint64), g


def check_detectable_corrected(rep, taus, alpha, fixed=None):
    """A10: every injection whose error clears 4 tau (or is not finite) is among the
    located and corrected elements.  Returns (must-correct count, masked list)."""
    if fixed is None:
        fixed = {(r["row"], r["col"]) for r in rep.records if r["kind"] in (1, 2)}
    big, masked = 0, []
    for g, tau in zip(rep.inject_log, taus):
        d = abs(g["new_val"] - g["old_val"]) * abs(alpha)
        if not np.isfinite(d) or d >= 4.0 * tau:
            big += 1
            assert (g["row"], g["col"]) in fixed, (g, tau)
        elif (g["row"], g["col"]) not in fixed:
            masked.append(g)
    return big, masked


def acc32_fault_taus(a, b, alpha, log, lam, bm=128, bn=128):
    """Binary32-path threshold of each injected element (beta = 0): the larger of
    its tile row's and tile column's, 2 lam sqrt(k + len + 8) u32 M with the
    magnitude bounds M_i = |alpha| (sum_p |a_ip|) max_p (sum_{j in J} |b_pj|) and
    M_j = |alpha| (sum_p |b_pj|) max_p (sum_{i in I} |a_ip|).  a = op(A), b = op(B)
    as (m x k) and (k x n) arrays of exact values."""
    import oracle
    a = np.abs(a)
    b = np.abs(b)
    m, k = a.shape
    n = b.shape[1]
    out = []
    for g in log:
        i, j = g["row"], g["col"]
        i0, j0 = (i // bm) * bm, (j // bn) * bn
        R, Q = min(bm, m - i0), min(bn, n - j0)
        mr = abs(alpha) * a[i, :].sum() * b[:, j0:j0 + Q].sum(axis=1).max()
        mc = abs(alpha) * b[:, j].sum() * a[i0:i0 + R, :].sum(axis=0).max()
        out.append(max(oracle.tau(k + Q + 8, mr, acc32=True, lam=lam),
                       oracle.tau(k + R + 8, mc, acc32=True, lam=lam)))
    return out
