"""GPU parity of the duplicated-computation (DMR) routines of §4 -- FT-DSCAL,
FT-DNRM2, FT-DGEMV, FT-DTRSV -- through the C ABI, against the CPU oracle's
plain BLAS definitions.

Bars: DSCAL is one product per element, so bitwise; DNRM2 within the rounding
bound of a sum of squares (bitwise on closed forms, including far outside the
range of unscaled squares); DGEMV within 2 gamma_{n+2} (|alpha||op(A)||x| +
|beta||y|) per element (bitwise on integer data); DTRSV within the forward
bound of a well-conditioned triangle (bitwise on integer solutions).  Under
injection every fault must be detected and corrected and the output must be
bitwise the fault-free one; a fault that repeats in the recomputation must end
uncorrectable."""
import math

import numpy as np
import pytest

import oracle
from tests.gpu_util import assert_close_f64

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2104_00897_amd import ftgemm
    assert torch.cuda.is_available()
    h = ftgemm.Handle(capacity=4096)
    yield ftgemm, h, torch
    torch.cuda.synchronize()
    h.close()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    return t.cpu().numpy()


def vec_positions(n, inc):
    pos = np.arange(n) * abs(inc)
    return pos[::-1].copy() if inc < 0 else pos


def flip(v, bit):
    return float(oracle.flip64(v, bit))


def check_log(rep, n_faults, lo=40, hi=63):
    assert rep.injected == n_faults and len(rep.inject_log) == n_faults
    for e in rep.inject_log:
        assert lo <= e["bit"] <= hi
        assert np.float64(e["new_val"]).view(np.uint64) == np.float64(flip(e["old_val"], e["bit"])).view(np.uint64)


# ------------------------------------------------------------------ DSCAL

@pytest.mark.parametrize("n", [1, 63, 511, 512, 513, 4097, 100003])
@pytest.mark.parametrize("incx", [1, 3])
@pytest.mark.parametrize("abft", [True, False])
def test_dscal_bitwise(env, n, incx, abft):
    ftgemm, h, torch = env
    rng = np.random.default_rng(n + incx)
    buf = rng.standard_normal(1 + (n - 1) * incx)
    d = dev(torch, buf)
    h.reset()
    ftgemm.dscal_f64(h, d, -1.7, n=n, incx=incx, cfg=ftgemm.make_config(abft=abft))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(d), oracle.dscal(buf, n, -1.7, incx))
    assert h.read().detected == 0


def test_dscal_unaligned_and_odd_lengths(env):
    """A vector starting 8 bytes past a 16-byte boundary (the one-element path)
    and lengths that end inside a run, against the 16-byte path's results."""
    ftgemm, h, torch = env
    rng = np.random.default_rng(77)
    for n in (1, 2, 511, 513, 1025, 100001):
        buf = rng.standard_normal(n + 1)
        d = dev(torch, buf)
        h.reset()
        ftgemm.dscal_f64(h, d[1:], 0.375, n=n)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(d), np.concatenate([buf[:1], oracle.dscal(buf[1:], n, 0.375)]))
        ftgemm.dscal_f64(h, d[1:], 2.0, n=n, cfg=ftgemm.make_config(seed=n, n_faults=min(n, 5)))
        torch.cuda.synchronize()
        rep = h.read()
        assert rep.injected == min(n, 5) and rep.corrected_recompute == min(n, 5)


def test_dscal_quick_returns_and_specials(env):
    ftgemm, h, torch = env
    buf = np.array([1.0, np.nan, np.inf, -0.0, 5.0])
    for n, inc in ((0, 1), (5, 0), (5, -1), (-3, 1)):
        d = dev(torch, buf)
        ftgemm.dscal_f64(h, d, 2.0, n=n, incx=inc)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(d), buf)
    d = dev(torch, buf)
    ftgemm.dscal_f64(h, d, 0.0, n=5)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(d), oracle.dscal(buf, 5, 0.0))


@pytest.mark.parametrize("target", ["acc", "checksum"])
def test_dscal_injected_faults_corrected(env, target):
    ftgemm, h, torch = env
    n = 100003
    rng = np.random.default_rng(5)
    buf = rng.standard_normal(n)
    ref = oracle.dscal(buf, n, 3.25)
    tg = ftgemm.TARGET_ACC if target == "acc" else ftgemm.TARGET_CHECKSUM
    d = dev(torch, buf)
    h.reset()
    ftgemm.dscal_f64(h, d, 3.25, cfg=ftgemm.make_config(seed=11, n_faults=20, target=tg, bit_lo=0, bit_hi=63))
    torch.cuda.synchronize()
    rep = h.read()
    np.testing.assert_array_equal(host(d), ref)
    check_log(rep, 20, 0, 63)
    assert rep.detected == 20 and rep.corrected_recompute == 20 and rep.uncorrectable == 0
    rows = sorted(e["row"] for e in rep.inject_log)
    assert len(set(rows)) == 20 and all(0 <= r < n for r in rows)
    assert sorted(r["row"] for r in rep.records) == rows
    assert all(r["kind"] == ftgemm.KIND_RECOMPUTE for r in rep.records)
    if target == "acc":
        # the flipped value is the product the oracle forms at that element
        for e in rep.inject_log:
            assert e["old_val"] == ref[e["row"]]


def test_dscal_persistent_fault_uncorrectable(env):
    ftgemm, h, torch = env
    n = 5000
    buf = np.random.default_rng(6).standard_normal(n)
    ref = oracle.dscal(buf, n, 2.5)
    d = dev(torch, buf)
    h.reset()
    ftgemm.dscal_f64(h, d, 2.5, cfg=ftgemm.make_config(seed=4, n_faults=5, target=ftgemm.TARGET_TWO_IN_SLOT))
    torch.cuda.synchronize()
    rep = h.read()
    assert rep.status == ftgemm.ERR_UNCORRECTED
    assert rep.injected == 5 and rep.detected == 5 and rep.uncorrectable == 5 and rep.corrected_recompute == 0
    out = host(d)
    bad = {e["row"]: e for e in rep.inject_log}
    for i, e in bad.items():
        assert out[i] == flip(ref[i], e["bit"])
    keep = np.ones(n, bool)
    keep[list(bad)] = False
    np.testing.assert_array_equal(out[keep], ref[keep])


def test_dscal_too_many_faults_unsupported(env):
    ftgemm, h, torch = env
    d = dev(torch, np.ones(1000))
    with pytest.raises(ftgemm.FtgError) as ei:
        ftgemm.dscal_f64(h, d, 2.0, cfg=ftgemm.make_config(seed=1, n_faults=65))
    assert ei.value.status == ftgemm.ERR_UNSUPPORTED


# ------------------------------------------------------------------ DNRM2

def nrm2(ftgemm, h, torch, buf, n=None, incx=1, cfg=None):
    d = dev(torch, buf)
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    ftgemm.dnrm2_f64(h, d, out, n=n, incx=incx, cfg=cfg)
    torch.cuda.synchronize()
    return float(out.item())


def nrm2_bound(n):
    """Relative bound of a sum of n non-negative squares in any order, the
    square root, and the few roundings of combining the scaled sums."""
    g = (n + 1) * U / (1 - (n + 1) * U)
    return 0.5 * g + 8 * U


@pytest.mark.parametrize("n", [1, 2, 100, 511, 513, 4096, 100003, 1048576 + 37])
@pytest.mark.parametrize("incx", [1, 2])
@pytest.mark.parametrize("abft", [True, False])
def test_dnrm2_matches_oracle(env, n, incx, abft):
    ftgemm, h, torch = env
    rng = np.random.default_rng(n * 3 + incx)
    buf = rng.standard_normal(1 + (n - 1) * incx) * 3.0
    got = nrm2(ftgemm, h, torch, buf, n, incx, ftgemm.make_config(abft=abft))
    ref = oracle.dnrm2(buf, n, incx)
    assert abs(got - ref) <= nrm2_bound(n) * ref


def test_dnrm2_unaligned(env):
    """The one-element path (a vector 8 bytes past a 16-byte boundary)."""
    ftgemm, h, torch = env
    rng = np.random.default_rng(78)
    for n in (3, 777, 100001):
        buf = rng.standard_normal(n + 1)
        d = dev(torch, buf)
        out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        ftgemm.dnrm2_f64(h, d[1:], out, n=n)
        torch.cuda.synchronize()
        ref = oracle.dnrm2(buf[1:], n)
        assert abs(float(out.item()) - ref) <= nrm2_bound(n) * ref


@pytest.mark.parametrize("e", [0, 600, -600, -1070, 1000])
def test_dnrm2_closed_forms_bitwise(env, e):
    """(3, 4, 12) 2^e: norm 13 2^e exactly, including where unscaled squares
    over- or underflow."""
    ftgemm, h, torch = env
    s = 2.0 ** e
    assert nrm2(ftgemm, h, torch, np.array([3.0 * s, 4.0 * s, 12.0 * s])) == 13.0 * s


def test_dnrm2_mixed_magnitudes(env):
    """Elements in all three of Blue's ranges at once (and long enough to span
    many workgroups)."""
    ftgemm, h, torch = env
    rng = np.random.default_rng(9)
    n = 300000
    buf = rng.standard_normal(n)
    buf[rng.integers(0, n, 50)] *= 2.0 ** 700
    buf[rng.integers(0, n, 5000)] *= 2.0 ** -700
    ref = oracle.dnrm2(buf, n)
    got = nrm2(ftgemm, h, torch, buf)
    assert abs(got - ref) <= nrm2_bound(n) * ref
    small = rng.standard_normal(n) * 2.0 ** -600
    small[::7] *= 2.0 ** 400
    ref = oracle.dnrm2(small, n)
    assert abs(nrm2(ftgemm, h, torch, small) - ref) <= nrm2_bound(n) * ref


def test_dnrm2_special_values(env):
    ftgemm, h, torch = env
    assert math.isnan(nrm2(ftgemm, h, torch, np.array([1.0, np.nan, np.inf])))
    assert nrm2(ftgemm, h, torch, np.array([1.0, -np.inf, 2.0])) == math.inf
    big = np.full(10000, 1.0)
    big[777] = np.nan
    assert math.isnan(nrm2(ftgemm, h, torch, big))
    assert nrm2(ftgemm, h, torch, np.zeros(1000)) == 0.0
    assert nrm2(ftgemm, h, torch, np.array([3.0, 4.0]), n=0) == 0.0
    assert nrm2(ftgemm, h, torch, np.array([3.0, 4.0]), n=2, incx=0) == 0.0
    assert nrm2(ftgemm, h, torch, np.array([3.0, 9.0, 4.0]), n=2, incx=2) == 5.0


@pytest.mark.parametrize("target", ["acc", "checksum"])
def test_dnrm2_injected_faults_corrected(env, target):
    ftgemm, h, torch = env
    n = 250007
    buf = np.random.default_rng(12).standard_normal(n)
    buf[::1000] *= 2.0 ** 600
    clean = nrm2(ftgemm, h, torch, buf)
    tg = ftgemm.TARGET_ACC if target == "acc" else ftgemm.TARGET_CHECKSUM
    h.reset()
    got = nrm2(ftgemm, h, torch, buf, cfg=ftgemm.make_config(seed=21, n_faults=20, target=tg, bit_lo=0, bit_hi=63))
    rep = h.read()
    assert np.float64(got).view(np.uint64) == np.float64(clean).view(np.uint64)
    check_log(rep, 20, 0, 63)
    assert rep.detected == 20 and rep.corrected_recompute == 20 and rep.uncorrectable == 0


def test_dnrm2_persistent_fault_uncorrectable(env):
    ftgemm, h, torch = env
    buf = np.random.default_rng(13).standard_normal(20000)
    h.reset()
    nrm2(ftgemm, h, torch, buf, cfg=ftgemm.make_config(seed=2, n_faults=3, target=ftgemm.TARGET_TWO_IN_SLOT))
    rep = h.read()
    assert rep.status == ftgemm.ERR_UNCORRECTED and rep.uncorrectable == 3 and rep.injected == 3


# ------------------------------------------------------------------ DGEMV

def gemv_case(ftgemm, h, torch, A, xb, yb, alpha, beta, ta, incx, incy, cfg=None):
    dA = ftgemm.to_device(A)
    dx, dy = dev(torch, xb), dev(torch, yb)
    ftgemm.dgemv_f64(h, dA, dx, dy, alpha, beta, ta, incx, incy, cfg)
    torch.cuda.synchronize()
    return host(dy)


def gemv_bound_check(A, xb, yb, out, ref, alpha, beta, ta, incx, incy):
    m, n = A.shape
    lenx, leny = (m, n) if ta else (n, m)
    px, py = vec_positions(lenx, incx), vec_positions(leny, incy)
    op = np.abs(A.T if ta else A)
    M = abs(alpha) * (op @ np.abs(xb[px]))
    if beta != 0.0:
        M = M + abs(beta) * np.abs(yb[py])
    assert_close_f64(out[py][:, None], ref[py][:, None], M[:, None], lenx + 2)
    untouched = np.ones(out.size, bool)
    untouched[py] = False
    np.testing.assert_array_equal(out[untouched], yb[untouched])


@pytest.mark.parametrize("ta", [0, 1])
@pytest.mark.parametrize("m,n", [(1, 1), (63, 65), (64, 64), (257, 1031), (3000, 40), (40, 3000)])
@pytest.mark.parametrize("incx,incy", [(1, 1), (-2, 3)])
def test_dgemv_matches_oracle(env, ta, m, n, incx, incy):
    ftgemm, h, torch = env
    rng = np.random.default_rng(m * 7 + n + ta)
    A = np.asfortranarray(rng.uniform(-1, 1, (m, n)))
    lenx, leny = (m, n) if ta else (n, m)
    xb = rng.uniform(-1, 1, 1 + (lenx - 1) * abs(incx))
    yb = rng.uniform(-1, 1, 1 + (leny - 1) * abs(incy))
    for alpha, beta in ((1.0, 0.0), (-0.75, 1.25)):
        ref = oracle.dgemv(A, xb, yb, alpha, beta, ta, incx, incy)
        h.reset()
        out = gemv_case(ftgemm, h, torch, A, xb, yb, alpha, beta, ta, incx, incy)
        gemv_bound_check(A, xb, yb, out, ref, alpha, beta, ta, incx, incy)
        assert h.read().detected == 0


@pytest.mark.parametrize("ta", [0, 1])
@pytest.mark.parametrize("m,n", [(64, 100000), (100000, 3), (5, 200003), (200003, 5)])
def test_dgemv_chunked_reduction(env, ta, m, n):
    """Shapes whose reduction is cut into many chunks (second pass)."""
    ftgemm, h, torch = env
    rng = np.random.default_rng(m + n + 5 * ta)
    A = np.asfortranarray(rng.uniform(-1, 1, (m, n)))
    lenx, leny = (m, n) if ta else (n, m)
    xb, yb = rng.uniform(-1, 1, lenx), rng.uniform(-1, 1, leny)
    for abft in (True, False):
        ref = oracle.dgemv(A, xb, yb, 2.0, -1.0, ta)
        out = gemv_case(ftgemm, h, torch, A, xb, yb, 2.0, -1.0, ta, 1, 1, ftgemm.make_config(abft=abft))
        gemv_bound_check(A, xb, yb, out, ref, 2.0, -1.0, ta, 1, 1)


@pytest.mark.parametrize("ta", [0, 1])
def test_dgemv_integer_bitwise(env, ta):
    ftgemm, h, torch = env
    rng = np.random.default_rng(40 + ta)
    m, n = 777, 1500
    A = np.asfortranarray(rng.integers(-8, 9, (m, n)).astype(np.float64))
    lenx, leny = (m, n) if ta else (n, m)
    xb = rng.integers(-8, 9, lenx).astype(np.float64)
    yb = rng.integers(-8, 9, leny).astype(np.float64)
    out = gemv_case(ftgemm, h, torch, A, xb, yb, 2.0, -3.0, ta, 1, 1)
    np.testing.assert_array_equal(out, oracle.dgemv(A, xb, yb, 2.0, -3.0, ta))


def test_dgemv_alpha_beta_special_cases(env):
    """beta = 0 does not read y (NaN ignored); alpha = 0 reads neither A nor x
    (NaN there) and scales y; alpha = 0, beta = 1 leaves y; alpha = beta = 0
    zeroes y."""
    ftgemm, h, torch = env
    rng = np.random.default_rng(41)
    m, n = 300, 200
    A = np.asfortranarray(rng.uniform(-1, 1, (m, n)))
    xb = rng.uniform(-1, 1, n)
    ynan = np.full(m, np.nan)
    out = gemv_case(ftgemm, h, torch, A, xb, ynan, 1.5, 0.0, 0, 1, 1)
    assert np.all(np.isfinite(out))
    Anan = np.full((m, n), np.nan, order="F")
    xnan = np.full(n, np.nan)
    yb = rng.uniform(-1, 1, 2 * m - 1)
    out = gemv_case(ftgemm, h, torch, Anan, xnan, yb, 0.0, 3.0, 0, 1, -2)
    np.testing.assert_array_equal(out, oracle.dgemv(Anan, xnan, yb, 0.0, 3.0, 0, 1, -2))
    out = gemv_case(ftgemm, h, torch, Anan, xnan, yb, 0.0, 1.0, 0, 1, 1)
    np.testing.assert_array_equal(out, yb)
    out = gemv_case(ftgemm, h, torch, Anan, xnan, ynan, 0.0, 0.0, 0, 1, 1)
    np.testing.assert_array_equal(out, np.zeros(m))


def test_dgemv_argument_errors(env):
    ftgemm, h, torch = env
    dA = ftgemm.to_device(np.ones((4, 4), order="F"))
    dx = dev(torch, np.ones(4))
    cases = [((2, 4, 4, 1.0, 4, 1, 0.0, 1), 1), ((0, -1, 4, 1.0, 4, 1, 0.0, 1), 2),
             ((0, 4, -1, 1.0, 4, 1, 0.0, 1), 3), ((0, 4, 4, 1.0, 3, 1, 0.0, 1), 6),
             ((0, 4, 4, 1.0, 4, 0, 0.0, 1), 8), ((0, 4, 4, 1.0, 4, 1, 0.0, 0), 11)]
    for (ta, m, n, alpha, lda, incx, beta, incy), info in cases:
        with pytest.raises(ftgemm.FtgError) as ei:
            h.dgemv(ta, m, n, alpha, ftgemm.ptr(dA), lda, ftgemm.ptr(dx), incx, beta, ftgemm.ptr(dx), incy)
        assert ei.value.status == ftgemm.ERR_INVALID_ARG and ei.value.info == info


@pytest.mark.parametrize("ta", [0, 1])
@pytest.mark.parametrize("target", ["acc", "checksum"])
@pytest.mark.parametrize("m,n", [(1000, 1100), (64, 100000)])
def test_dgemv_injected_faults_corrected(env, ta, target, m, n):
    ftgemm, h, torch = env
    rng = np.random.default_rng(50 + ta)
    A = np.asfortranarray(rng.uniform(-1, 1, (m, n)))
    lenx, leny = (m, n) if ta else (n, m)
    xb, yb = rng.uniform(-1, 1, lenx), rng.uniform(-1, 1, leny)
    clean = gemv_case(ftgemm, h, torch, A, xb, yb, 1.0, 0.5, ta, 1, 1)
    tg = ftgemm.TARGET_ACC if target == "acc" else ftgemm.TARGET_CHECKSUM
    h.reset()
    out = gemv_case(ftgemm, h, torch, A, xb, yb, 1.0, 0.5, ta, 1, 1,
                    ftgemm.make_config(seed=31 + ta, n_faults=20, target=tg, bit_lo=0, bit_hi=63))
    rep = h.read()
    np.testing.assert_array_equal(out, clean)
    check_log(rep, 20, 0, 63)
    assert rep.detected == 20 and rep.corrected_recompute == 20 and rep.uncorrectable == 0
    for e in rep.inject_log:
        if ta:
            assert 0 <= e["row"] < m and 0 <= e["col"] < n
        else:
            assert 0 <= e["row"] < m and 0 <= e["col"] < n and e["col"] % 8 == 0


def test_dgemv_persistent_fault_uncorrectable(env):
    ftgemm, h, torch = env
    rng = np.random.default_rng(52)
    A = np.asfortranarray(rng.uniform(-1, 1, (500, 600)))
    xb, yb = rng.uniform(-1, 1, 600), rng.uniform(-1, 1, 500)
    h.reset()
    gemv_case(ftgemm, h, torch, A, xb, yb, 1.0, 0.0, 0, 1, 1,
              ftgemm.make_config(seed=8, n_faults=4, target=ftgemm.TARGET_TWO_IN_SLOT))
    rep = h.read()
    assert rep.status == ftgemm.ERR_UNCORRECTED and rep.uncorrectable == 4 and rep.injected == 4


def test_dgemv_full_size_sampled(env):
    """16384^2 without transpose and transposed in the launch shape the bench
    times: 4096 sampled outputs against the oracle on the sampled rows (or
    columns) of A."""
    ftgemm, h, torch = env
    n = 16384
    g = torch.Generator(device="cuda").manual_seed(3)
    dA = torch.rand((n, n), generator=g, device="cuda", dtype=torch.float64) * 2 - 1
    dx = torch.rand(n, generator=g, device="cuda", dtype=torch.float64) * 2 - 1
    dy0 = torch.rand(n, generator=g, device="cuda", dtype=torch.float64) * 2 - 1
    pick = np.sort(np.random.default_rng(4).choice(n, 4096, replace=False))
    xb, yb = host(dx), host(dy0)
    for ta in (0, 1):
        dy = dy0.clone()
        h.reset()
        ftgemm.dgemv_f64(h, dA, dx, dy, 1.0, 0.5, ta)
        torch.cuda.synchronize()
        assert h.read().detected == 0
        # column-major A(i, j) is dA[j, i]: rows of A are columns of dA
        idx = torch.from_numpy(pick).cuda()
        # the sampled rows of op(A): rows of A are dA[:, i], columns of A are dA[j, :]
        sub = np.asfortranarray(host(dA[idx, :]) if ta else host(dA[:, idx]).T)
        ref = oracle.dgemv(sub, xb, yb[pick], 1.0, 0.5, 0)
        M = np.abs(sub) @ np.abs(xb) + 0.5 * np.abs(yb[pick])
        assert_close_f64(host(dy)[pick][:, None], ref[:, None], M[:, None], n + 2)
    del dA


# ------------------------------------------------------------------ DTRSV

def tri_op(A, uplo, ta, diag):
    T = np.tril(A) if uplo == 0 else np.triu(A)
    if diag:
        np.fill_diagonal(T, 1.0)
    return T.T if ta else T


def hide(A, uplo, diag):
    X = A.copy(order="F")
    n = A.shape[0]
    X[np.triu_indices(n, 1) if uplo == 0 else np.tril_indices(n, -1)] = np.nan
    if diag:
        np.fill_diagonal(X, np.nan)
    return X


def well_conditioned(rng, n):
    """Diagonal in [1, 2], off-diagonal U[-1, 1] * 0.5 / n: every triangle of it
    has an inverse of norm at most 2, so the forward error is a few times the
    backward error gamma_n."""
    A = rng.uniform(-1, 1, (n, n)) * (0.5 / n)
    np.fill_diagonal(A, rng.uniform(1, 2, n))
    return np.asfortranarray(A)


def trsv_case(ftgemm, h, torch, A, xb, uplo, ta, diag, incx, cfg=None):
    dA = ftgemm.to_device(A)
    dx = dev(torch, xb)
    ftgemm.dtrsv_f64(h, dA, dx, uplo, ta, diag, incx, cfg)
    torch.cuda.synchronize()
    return host(dx)


@pytest.mark.parametrize("uplo", [0, 1])
@pytest.mark.parametrize("ta", [0, 1])
@pytest.mark.parametrize("diag", [0, 1])
@pytest.mark.parametrize("n,incx", [(1, 1), (127, 1), (128, -2), (129, 1), (300, 3), (1000, 1)])
def test_dtrsv_matches_oracle(env, uplo, ta, diag, n, incx):
    ftgemm, h, torch = env
    rng = np.random.default_rng(n * 8 + 4 * uplo + 2 * ta + diag)
    A = hide(well_conditioned(rng, n), uplo, diag)
    xb = rng.uniform(-1, 1, 1 + (n - 1) * abs(incx))
    ref = oracle.dtrsv(A, xb, uplo, ta, diag, incx)
    for abft in (True, False):
        h.reset()
        out = trsv_case(ftgemm, h, torch, A, xb, uplo, ta, diag, incx, ftgemm.make_config(abft=abft))
        pos = vec_positions(n, incx)
        bound = 16 * (n + 2) * U * (1.0 + np.max(np.abs(ref[pos])))
        assert np.max(np.abs(out[pos] - ref[pos])) <= bound
        keep = np.ones(xb.size, bool)
        keep[pos] = False
        np.testing.assert_array_equal(out[keep], xb[keep])
        assert h.read().detected == 0


@pytest.mark.parametrize("uplo", [0, 1])
@pytest.mark.parametrize("ta", [0, 1])
@pytest.mark.parametrize("diag", [0, 1])
def test_dtrsv_integer_solution_bitwise(env, uplo, ta, diag):
    """Integer x and b = op(T) x with small integers off the diagonal and a
    power-of-two diagonal (whose reciprocals are exact): every step is exact,
    so the solve returns x bitwise across several blocks."""
    ftgemm, h, torch = env
    rng = np.random.default_rng(300 + 4 * uplo + 2 * ta + diag)
    n = 333
    A = rng.integers(-1, 2, size=(n, n)).astype(np.float64)
    np.fill_diagonal(A, rng.choice([-2.0, -1.0, 1.0, 2.0], size=n))
    T = tri_op(A, uplo, ta, diag)
    x = rng.integers(-3, 4, size=n).astype(np.float64)
    # keep every partial sum exact: entries of b and of each step stay small integers
    b = T @ x
    out = trsv_case(ftgemm, h, torch, hide(np.asfortranarray(A), uplo, diag), b, uplo, ta, diag, 1)
    ref = oracle.dtrsv(hide(np.asfortranarray(A), uplo, diag), b, uplo, ta, diag, 1)
    np.testing.assert_array_equal(ref, x)
    np.testing.assert_array_equal(out, x)


@pytest.mark.parametrize("uplo,ta", [(0, 0), (1, 1), (1, 0)])
@pytest.mark.parametrize("target", ["acc", "checksum"])
def test_dtrsv_injected_faults_corrected(env, uplo, ta, target):
    ftgemm, h, torch = env
    n = 1000
    rng = np.random.default_rng(60 + uplo + 2 * ta)
    A = hide(well_conditioned(rng, n), uplo, 0)
    xb = rng.uniform(-1, 1, n)
    clean = trsv_case(ftgemm, h, torch, A, xb, uplo, ta, 0, 1)
    tg = ftgemm.TARGET_ACC if target == "acc" else ftgemm.TARGET_CHECKSUM
    h.reset()
    out = trsv_case(ftgemm, h, torch, A, xb, uplo, ta, 0, 1,
                    ftgemm.make_config(seed=70 + uplo, n_faults=20, target=tg, bit_lo=0, bit_hi=63))
    rep = h.read()
    np.testing.assert_array_equal(out, clean)
    check_log(rep, 20, 0, 63)
    assert rep.detected == 20 and rep.corrected_recompute == 20 and rep.uncorrectable == 0
    assert {e["interval"] for e in rep.inject_log} <= {0, 1}
    assert all(0 <= e["row"] < n for e in rep.inject_log)


def test_dtrsv_persistent_fault_uncorrectable(env):
    ftgemm, h, torch = env
    n = 400
    rng = np.random.default_rng(64)
    A = hide(well_conditioned(rng, n), 0, 0)
    h.reset()
    trsv_case(ftgemm, h, torch, A, rng.uniform(-1, 1, n), 0, 0, 0, 1,
              ftgemm.make_config(seed=5, n_faults=6, target=ftgemm.TARGET_TWO_IN_SLOT))
    rep = h.read()
    assert rep.status == ftgemm.ERR_UNCORRECTED and rep.uncorrectable == 6 and rep.injected == 6


def test_dtrsv_argument_errors(env):
    ftgemm, h, torch = env
    dA = ftgemm.to_device(np.eye(4, order="F"))
    dx = dev(torch, np.ones(4))
    cases = [((2, 0, 0, 4, 4, 1), 1), ((0, 2, 0, 4, 4, 1), 2), ((0, 0, 2, 4, 4, 1), 3),
             ((0, 0, 0, -1, 4, 1), 4), ((0, 0, 0, 4, 3, 1), 6), ((0, 0, 0, 4, 4, 0), 8)]
    for (uplo, ta, diag, n, lda, incx), info in cases:
        with pytest.raises(ftgemm.FtgError) as ei:
            h.dtrsv(uplo, ta, diag, n, ftgemm.ptr(dA), lda, ftgemm.ptr(dx), incx)
        assert ei.value.status == ftgemm.ERR_INVALID_ARG and ei.value.info == info


def test_dtrsv_full_size_residual(env):
    """n = 16384 (lower, no transpose, the bench's launch shape): the residual
    of the computed solution satisfies the substitution's backward bound
    |b - T x| <= gamma_{n+2} |T| |x| (times 2 for the reciprocal products)."""
    ftgemm, h, torch = env
    n = 16384
    rng = np.random.default_rng(65)
    A = well_conditioned(rng, n)
    b = rng.uniform(-1, 1, n)
    out = trsv_case(ftgemm, h, torch, A, b, 0, 0, 0, 1)
    T = np.tril(A)
    g = (n + 2) * U / (1 - (n + 2) * U)
    assert np.all(np.abs(b - T @ out) <= 2 * g * (np.abs(T) @ np.abs(out)) + 1e-300)
