"""CPU oracle for the checksum-protected GEMM -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` import this package.  The GPU library (``paper_2104_00897_amd``)
never imports it and shares no code with it.

The arithmetic lives in ``ftgemm_oracle.c`` (plain C, binary64, built with
``-O2 -ffp-contract=off``); this module builds it with gcc and wraps it with
ctypes, taking and returning numpy arrays in Fortran (column-major) order.

Functions and the passages of the paper (Zhai et al., FT-BLAS, ICS'21) they follow:
  gemm          C := alpha op(A) op(B) + beta C            (§2.1, §3.3.2)
  gemm_entries  selected entries of the same               (sampled checks)
  abft          per-tile online ABFT: encode, maintain,    (§2.1, §5.1, §5.2, §6.3)
                verify, locate, correct
  fault_plan    seeded injection plan                      (§6.3)
  flip64/flip32 single-bit flips of a value                (fault model, §1)
  splitmix64    counter-based generator (Steele et al. 2014)
  tau / gamma   round-off threshold (reading of §2.1's "round-off threshold")
  dsymm / dtrmm the Level-3 routines of §6.2.3 that run on the protected
  / dtrsm       product, by their plain definitions (dtrsm: substitution)
  dscal / dnrm2 the Level-1/2 routines protected by duplicated computation
  / dgemv       (§3.1, §3.2, §4), by their plain BLAS definitions (dnrm2:
  / dtrsv       exact power-of-two scaling; dtrsv: substitution)
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ftgemm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libftgemm_oracle.so")
_lib = None

KIND_SUBTRACT = 1
KIND_RECOMPUTE = 2
KIND_CHECKSUM_ONLY = 3
KIND_UNCORRECTABLE = 4
KIND_TILE_RECOMPUTED = 5

TARGET_ACC = 0
TARGET_CHECKSUM = 1
TARGET_TWO_IN_SLOT = 2


def build() -> str:
    """Compile the oracle with gcc (always recompiles). Returns the library path."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c11",
           "-Wall", "-shared", "-fPIC", "-o", _LIB_PATH, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB_PATH


class _Fault(ct.Structure):
    _fields_ = [("tile_m", ct.c_int64), ("tile_n", ct.c_int64), ("interval", ct.c_int64),
                ("row", ct.c_int64), ("col", ct.c_int64), ("pflip", ct.c_int64),
                ("bit", ct.c_int32), ("target", ct.c_int32)]


class _Params(ct.Structure):
    _fields_ = [("ta", ct.c_int32), ("tb", ct.c_int32),
                ("m", ct.c_int64), ("n", ct.c_int64), ("k", ct.c_int64),
                ("alpha", ct.c_double), ("beta", ct.c_double),
                ("lda", ct.c_int64), ("ldb", ct.c_int64), ("ldc", ct.c_int64),
                ("bm", ct.c_int64), ("bn", ct.c_int64), ("kc", ct.c_int64),
                ("acc32", ct.c_int32), ("lam", ct.c_double),
                ("correct_policy", ct.c_int32), ("uncorrectable_policy", ct.c_int32),
                ("split", ct.c_int32)]


class _Record(ct.Structure):
    _fields_ = [("tile_m", ct.c_int64), ("tile_n", ct.c_int64), ("interval", ct.c_int64),
                ("row", ct.c_int64), ("col", ct.c_int64), ("kind", ct.c_int32),
                ("delta", ct.c_double), ("tau", ct.c_double)]


class _Counts(ct.Structure):
    _fields_ = [("injected", ct.c_int64), ("detected", ct.c_int64),
                ("corrected_subtract", ct.c_int64), ("corrected_recompute", ct.c_int64),
                ("checksum_only", ct.c_int64), ("uncorrectable", ct.c_int64),
                ("tiles_recomputed", ct.c_int64), ("n_records", ct.c_int64)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ct.CDLL(_LIB_PATH)
    dp = ct.POINTER(ct.c_double)
    i64 = ct.c_int64
    lib.ftgo_gemm.argtypes = [ct.c_int, ct.c_int, i64, i64, i64, ct.c_double, dp, i64, dp, i64,
                              ct.c_double, dp, i64]
    lib.ftgo_gemm.restype = ct.c_int
    lib.ftgo_gemm_entries.argtypes = [ct.c_int, ct.c_int, i64, i64, i64, ct.c_double, dp, i64,
                                      dp, i64, ct.c_double, dp, i64, i64,
                                      ct.POINTER(i64), ct.POINTER(i64), dp]
    lib.ftgo_gemm_entries.restype = ct.c_int
    lib.ftgo_flip64.argtypes = [ct.c_double, ct.c_int]
    lib.ftgo_flip64.restype = ct.c_double
    lib.ftgo_flip32.argtypes = [ct.c_float, ct.c_int]
    lib.ftgo_flip32.restype = ct.c_float
    lib.ftgo_splitmix64.argtypes = [ct.c_uint64, ct.c_uint64]
    lib.ftgo_splitmix64.restype = ct.c_uint64
    lib.ftgo_slot_permutation.argtypes = [ct.c_uint64, ct.c_uint64, ct.POINTER(ct.c_uint64),
                                          ct.POINTER(ct.c_uint64)]
    lib.ftgo_slot_permutation.restype = None
    lib.ftgo_fault_plan.argtypes = [ct.c_uint64, i64, ct.c_int32, ct.c_int32, ct.c_int32,
                                    i64, i64, i64, i64, i64, i64, i64,
                                    ct.POINTER(_Fault), i64]
    lib.ftgo_fault_plan.restype = i64
    lib.ftgo_gamma.argtypes = [i64]
    lib.ftgo_gamma.restype = ct.c_double
    lib.ftgo_tau.argtypes = [ct.c_int, ct.c_double, i64, ct.c_double]
    lib.ftgo_tau.restype = ct.c_double
    lib.ftgo_abft.argtypes = [ct.POINTER(_Params), dp, dp, dp, ct.POINTER(_Fault), i64,
                              ct.POINTER(_Record), i64, ct.POINTER(_Counts)]
    lib.ftgo_abft.restype = ct.c_int
    lib.ftgo_dsymm.argtypes = [ct.c_int, ct.c_int, i64, i64, ct.c_double, dp, i64, dp, i64, ct.c_double,
                               dp, i64]
    lib.ftgo_dsymm.restype = ct.c_int
    lib.ftgo_dtrmm.argtypes = [ct.c_int, ct.c_int, ct.c_int, ct.c_int, i64, i64, ct.c_double, dp, i64,
                               dp, i64]
    lib.ftgo_dtrmm.restype = ct.c_int
    lib.ftgo_dtrsm.argtypes = lib.ftgo_dtrmm.argtypes
    lib.ftgo_dtrsm.restype = ct.c_int
    lib.ftgo_dscal.argtypes = [i64, ct.c_double, dp, i64]
    lib.ftgo_dscal.restype = None
    lib.ftgo_dnrm2.argtypes = [i64, dp, i64]
    lib.ftgo_dnrm2.restype = ct.c_double
    lib.ftgo_dgemv.argtypes = [ct.c_int, i64, i64, ct.c_double, dp, i64, dp, i64, ct.c_double, dp, i64]
    lib.ftgo_dgemv.restype = ct.c_int
    lib.ftgo_dtrsv.argtypes = [ct.c_int, ct.c_int, ct.c_int, i64, dp, i64, dp, i64]
    lib.ftgo_dtrsv.restype = ct.c_int
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _f64(a) -> np.ndarray:
    """Fortran-ordered binary64 copy (exact for bf16/fp8/fp32 inputs)."""
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def _ld(a: np.ndarray) -> int:
    return max(1, a.shape[0])


def gemm(A, B, C=None, alpha=1.0, beta=0.0, ta=0, tb=0):
    """Returns alpha*op(A)*op(B) + beta*C (C not read when beta == 0)."""
    A = _f64(A); B = _f64(B)
    m = A.shape[1] if ta else A.shape[0]
    k = A.shape[0] if ta else A.shape[1]
    n = B.shape[0] if tb else B.shape[1]
    C = np.zeros((m, n), order="F") if C is None else _f64(C).copy(order="F")
    info = _load().ftgo_gemm(ta, tb, m, n, k, alpha, _dptr(A), _ld(A), _dptr(B), _ld(B),
                             beta, _dptr(C), _ld(C))
    if info:
        raise ValueError(f"ftgo_gemm: invalid argument {info}")
    return C


def gemm_entries(A, B, C, rows, cols, alpha=1.0, beta=0.0, ta=0, tb=0):
    A = _f64(A); B = _f64(B)
    m = A.shape[1] if ta else A.shape[0]
    k = A.shape[0] if ta else A.shape[1]
    n = B.shape[0] if tb else B.shape[1]
    if C is None:
        C = np.zeros((1, 1), order="F")
        ldc = max(1, m)
    else:
        C = _f64(C)
        ldc = _ld(C)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.zeros(len(rows))
    i64p = ct.POINTER(ct.c_int64)
    info = _load().ftgo_gemm_entries(ta, tb, m, n, k, alpha, _dptr(A), _ld(A), _dptr(B), _ld(B),
                                     beta, _dptr(C), ldc, len(rows),
                                     rows.ctypes.data_as(i64p), cols.ctypes.data_as(i64p),
                                     _dptr(out))
    if info:
        raise ValueError(f"ftgo_gemm_entries: invalid argument {info}")
    return out


def flip64(x: float, bit: int) -> float:
    return _load().ftgo_flip64(x, bit)


def flip32(x: float, bit: int) -> float:
    return _load().ftgo_flip32(x, bit)


def splitmix64(seed: int, ctr: int) -> int:
    return _load().ftgo_splitmix64(seed & (2**64 - 1), ctr & (2**64 - 1))


def slot_permutation(seed: int, S: int):
    a = ct.c_uint64(); b = ct.c_uint64()
    _load().ftgo_slot_permutation(seed & (2**64 - 1), S, ct.byref(a), ct.byref(b))
    return a.value, b.value


def gamma(nterms: int) -> float:
    return _load().ftgo_gamma(nterms)


def tau(nterms: int, mag: float, acc32: bool = False, lam: float = 1.0) -> float:
    return _load().ftgo_tau(int(acc32), lam, nterms, mag)


@dataclass
class Fault:
    tile_m: int
    tile_n: int
    interval: int
    row: int      # tile-local
    col: int      # tile-local
    pflip: int    # global step after whose update the flip lands
    bit: int
    target: int


def fault_plan(seed, n_faults, m, n, k, bm, bn, kc=0, kgran=16, bit_lo=40, bit_hi=63,
               target=TARGET_ACC):
    cap = 2 * max(1, n_faults) + 2
    buf = (_Fault * cap)()
    w = _load().ftgo_fault_plan(seed & (2**64 - 1), n_faults, target, bit_lo, bit_hi, m, n, k,
                                bm, bn, kc, kgran, buf, cap)
    return [Fault(f.tile_m, f.tile_n, f.interval, f.row, f.col, f.pflip, f.bit, f.target)
            for f in buf[:w]]


@dataclass
class Record:
    tile_m: int
    tile_n: int
    interval: int
    row: int   # global, -1 if n/a
    col: int   # global, -1 if n/a
    kind: int
    delta: float
    tau: float


def abft(A, B, C=None, alpha=1.0, beta=0.0, ta=0, tb=0, bm=128, bn=128, kc=0, plan=(),
         acc32=False, lam=1.0, correct_policy=0, uncorrectable_policy=0, cap=4096, split=False):
    """Simulates the protected product; returns (C_out, records, counts dict).

    split: with intervals (kc), C is the accumulator from one interval to the
    next (the K_c loop of the blocked GEMM, §5.1): interval t is checked as the
    product C := alpha A_t B_t + beta_t C with its own accumulator, checksums and
    magnitudes, beta_t = beta for the first interval and 1 after; without it the
    accumulator runs on through the intervals (the online scheme of §2.1)."""
    A = _f64(A); B = _f64(B)
    m = A.shape[1] if ta else A.shape[0]
    k = A.shape[0] if ta else A.shape[1]
    n = B.shape[0] if tb else B.shape[1]
    C = np.zeros((m, n), order="F") if C is None else _f64(C).copy(order="F")
    P = _Params(ta, tb, m, n, k, alpha, beta, _ld(A), _ld(B), _ld(C), bm, bn, kc, int(acc32),
                lam, correct_policy, uncorrectable_policy, int(split))
    plan = list(plan)
    pa = (_Fault * max(1, len(plan)))()
    for q, f in enumerate(plan):
        pa[q] = _Fault(f.tile_m, f.tile_n, f.interval, f.row, f.col, f.pflip, f.bit, f.target)
    recs = (_Record * cap)()
    cnt = _Counts()
    info = _load().ftgo_abft(ct.byref(P), _dptr(A), _dptr(B), _dptr(C), pa, len(plan), recs, cap,
                             ct.byref(cnt))
    if info:
        raise ValueError(f"ftgo_abft: error {info}")
    records = [Record(r.tile_m, r.tile_n, r.interval, r.row, r.col, r.kind, r.delta, r.tau)
               for r in recs[:min(cap, cnt.n_records)]]
    counts = {f: getattr(cnt, f) for f, _ in _Counts._fields_}
    return C, records, counts


def dsymm(A, B, C=None, alpha=1.0, beta=0.0, side=0, uplo=0):
    """C := alpha A B + beta C (side 0) or alpha B A + beta C (side 1), A symmetric
    with only its lower (uplo 0) or upper (uplo 1) triangle read."""
    A = _f64(A); B = _f64(B)
    m, n = B.shape
    C = np.zeros((m, n), order="F") if C is None else _f64(C).copy(order="F")
    info = _load().ftgo_dsymm(side, uplo, m, n, alpha, _dptr(A), _ld(A), _dptr(B), _ld(B), beta,
                              _dptr(C), _ld(C))
    if info:
        raise ValueError(f"ftgo_dsymm: invalid argument {info}")
    return C


def dtrmm(A, B, alpha=1.0, side=0, uplo=0, ta=0, diag=0):
    """B := alpha op(A) B (side 0) or alpha B op(A) (side 1), A triangular (uplo 0
    lower, 1 upper; diag 1 = unit, diagonal not read); returns the new B."""
    A = _f64(A)
    B = _f64(B).copy(order="F")
    m, n = B.shape
    info = _load().ftgo_dtrmm(side, uplo, ta, diag, m, n, alpha, _dptr(A), _ld(A), _dptr(B), _ld(B))
    if info:
        raise ValueError(f"ftgo_dtrmm: invalid argument {info}")
    return B


def dtrsm(A, B, alpha=1.0, side=0, uplo=0, ta=0, diag=0):
    """B := alpha op(A)^-1 B (side 0) or alpha B op(A)^-1 (side 1) by substitution,
    A triangular (uplo 0 lower, 1 upper; diag 1 = unit); returns the new B."""
    A = _f64(A)
    B = _f64(B).copy(order="F")
    m, n = B.shape
    info = _load().ftgo_dtrsm(side, uplo, ta, diag, m, n, alpha, _dptr(A), _ld(A), _dptr(B), _ld(B))
    if info:
        raise ValueError(f"ftgo_dtrsm: invalid argument {info}")
    return B



def _vec(buf):
    """1-D float64 copy of a strided-vector buffer."""
    return np.ascontiguousarray(np.asarray(buf, dtype=np.float64).ravel()).copy()


def dscal(buf, n, alpha, incx=1):
    """x := alpha x over n elements of buf at stride incx (BLAS dscal); returns
    the new buffer."""
    x = _vec(buf)
    if n > 0 and incx > 0 and (n - 1) * incx >= x.size:
        raise ValueError("dscal: buffer too short")
    _load().ftgo_dscal(n, alpha, _dptr(x), incx)
    return x


def dnrm2(buf, n, incx=1):
    """Euclidean norm of n elements of buf at stride incx (BLAS dnrm2)."""
    x = _vec(buf)
    if n > 0 and incx > 0 and (n - 1) * incx >= x.size:
        raise ValueError("dnrm2: buffer too short")
    return float(_load().ftgo_dnrm2(n, _dptr(x), incx))


def dgemv(A, xbuf, ybuf, alpha=1.0, beta=0.0, ta=0, incx=1, incy=1):
    """y := alpha op(A) x + beta y (BLAS dgemv) on the vectors held in xbuf/ybuf
    at strides incx/incy (negative: element 0 at the far end); returns the new
    y buffer."""
    A = _f64(A)
    m, n = A.shape
    x, y = _vec(xbuf), _vec(ybuf)
    lenx, leny = (m, n) if ta else (n, m)
    if (lenx - 1) * abs(incx) >= max(x.size, 1) or (leny - 1) * abs(incy) >= max(y.size, 1):
        raise ValueError("dgemv: vector buffer too short")
    info = _load().ftgo_dgemv(ta, m, n, alpha, _dptr(A), _ld(A), _dptr(x), incx, beta, _dptr(y), incy)
    if info:
        raise ValueError(f"ftgo_dgemv: invalid argument {info}")
    return y


def dtrsv(A, xbuf, uplo=0, ta=0, diag=0, incx=1):
    """x := op(A)^-1 x (BLAS dtrsv) on the vector held in xbuf at stride incx;
    returns the new buffer."""
    A = _f64(A)
    n = A.shape[0]
    x = _vec(xbuf)
    if n and (n - 1) * abs(incx) >= x.size:
        raise ValueError("dtrsv: vector buffer too short")
    info = _load().ftgo_dtrsv(uplo, ta, diag, n, _dptr(A), _ld(A), _dptr(x), incx)
    if info:
        raise ValueError(f"ftgo_dtrsv: invalid argument {info}")
    return x
