"""ctypes binding of the protected-GEMM C ABI (include/ftgemm.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libftgemm.so.  torch provides device memory and the current
stream.  Matrices are column-major; a column-major (rows x cols) matrix is
held in a torch tensor of shape (cols, rows) (see ``to_device``/``to_host``).
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libftgemm.so")

OP_N, OP_T = 0, 1
LEFT, RIGHT = 0, 1
LOWER, UPPER = 0, 1
NON_UNIT, UNIT = 0, 1
F64, F32, BF16, F8_E4M3 = 0, 1, 2, 3
OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_HIP, ERR_UNCORRECTED = 0, 1, 2, 3, 4
KIND_SUBTRACT, KIND_RECOMPUTE, KIND_CHECKSUM_ONLY, KIND_UNCORRECTABLE, KIND_TILE_RECOMPUTED = 1, 2, 3, 4, 5
TARGET_ACC, TARGET_CHECKSUM, TARGET_TWO_IN_SLOT = 0, 1, 2
KGRAN = 128  # injection / interval granularity in k


class FtgError(RuntimeError):
    def __init__(self, status: int, what: str, info: int = 0):
        self.status = status
        self.info = info
        super().__init__(f"{what}: status {status}" + (f" (argument {info})" if info else ""))


class Inject(ct.Structure):
    _fields_ = [("seed", ct.c_uint64), ("n_faults", ct.c_uint32), ("target", ct.c_uint32),
                ("per_mac_rate", ct.c_double), ("bit_lo", ct.c_int32), ("bit_hi", ct.c_int32)]


class Config(ct.Structure):
    _fields_ = [("abft", ct.c_int32), ("interval_k", ct.c_int32), ("lam", ct.c_double),
                ("correct_policy", ct.c_int32), ("uncorrectable_policy", ct.c_int32),
                ("tile", ct.c_int32), ("encode_in_loop", ct.c_int32), ("inject", ct.POINTER(Inject))]


class FaultRecord(ct.Structure):
    _fields_ = [("problem", ct.c_int32), ("tile_m", ct.c_int32), ("tile_n", ct.c_int32),
                ("interval", ct.c_int32), ("row", ct.c_int64), ("col", ct.c_int64),
                ("kind", ct.c_int32), ("reserved", ct.c_int32), ("delta", ct.c_double),
                ("tau", ct.c_double)]


class InjectRecord(ct.Structure):
    _fields_ = [("problem", ct.c_int32), ("tile_m", ct.c_int32), ("tile_n", ct.c_int32),
                ("interval", ct.c_int32), ("row", ct.c_int64), ("col", ct.c_int64),
                ("pflip", ct.c_int64), ("bit", ct.c_int32), ("target", ct.c_int32),
                ("old_val", ct.c_double), ("new_val", ct.c_double)]


class FaultReport(ct.Structure):
    _fields_ = [("injected", ct.c_uint64), ("detected", ct.c_uint64),
                ("corrected_subtract", ct.c_uint64), ("corrected_recompute", ct.c_uint64),
                ("checksum_only", ct.c_uint64), ("uncorrectable", ct.c_uint64),
                ("tiles_recomputed", ct.c_uint64), ("n_records", ct.c_uint32),
                ("n_inject_log", ct.c_uint32), ("capacity", ct.c_uint32), ("lost", ct.c_uint32),
                ("max_pass_ratio", ct.c_double),
                ("records", ct.POINTER(FaultRecord)), ("inject_log", ct.POINTER(InjectRecord))]


EXPORTS = [
    "ftg_create", "ftg_destroy", "ftg_dgemm", "ftg_gemm_ex", "ftg_dgemm_batched_uneven",
    "ftg_batched_reserve", "ftg_report_read", "ftg_report_reset", "ftg_last_error_arg",
    "ftg_tile_info", "ftg_tune_set", "ftg_tune_get", "ftg_timing_enable", "ftg_timing_read",
    "ftg_status_string", "ftg_dgemm_noalloc", "ftg_dgemm_noalloc_max_bytes",
    "ftg_workspace_reserve", "ftg_default_lambda", "ftg_dgemm_unfused", "ftg_dsymm", "ftg_dtrmm",
    "ftg_dtrsm", "ftg_dscal", "ftg_dnrm2", "ftg_dgemv", "ftg_dtrsv",
]

_lib = None


def load() -> ct.CDLL:
    """Loads libftgemm.so (built by __graft_entry__.build / build.py); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FtgError(ERR_HIP, f"HIP library missing: {LIB_PATH} (run the build first)")
    lib = ct.CDLL(LIB_PATH)
    i64, vp, i32 = ct.c_int64, ct.c_void_p, ct.c_int32
    h = ct.c_void_p
    lib.ftg_create.argtypes = [ct.POINTER(h), ct.c_size_t]
    lib.ftg_destroy.argtypes = [h]
    lib.ftg_dgemm.argtypes = [h, i32, i32, i64, i64, i64, ct.c_double, vp, i64, vp, i64,
                              ct.c_double, vp, i64, vp, ct.POINTER(Config)]
    lib.ftg_dgemm_noalloc.argtypes = lib.ftg_dgemm.argtypes
    lib.ftg_dgemm_unfused.argtypes = lib.ftg_dgemm.argtypes
    lib.ftg_dsymm.argtypes = [h, i32, i32, i64, i64, ct.c_double, vp, i64, vp, i64, ct.c_double, vp,
                              i64, vp, ct.POINTER(Config)]
    lib.ftg_dtrmm.argtypes = [h, i32, i32, i32, i32, i64, i64, ct.c_double, vp, i64, vp, i64, vp,
                              ct.POINTER(Config)]
    lib.ftg_dtrsm.argtypes = lib.ftg_dtrmm.argtypes
    lib.ftg_dscal.argtypes = [h, i64, ct.c_double, vp, i64, vp, ct.POINTER(Config)]
    lib.ftg_dnrm2.argtypes = [h, i64, vp, i64, vp, vp, ct.POINTER(Config)]
    lib.ftg_dgemv.argtypes = [h, i32, i64, i64, ct.c_double, vp, i64, vp, i64, ct.c_double, vp, i64, vp,
                              ct.POINTER(Config)]
    lib.ftg_dtrsv.argtypes = [h, i32, i32, i32, i64, vp, i64, vp, i64, vp, ct.POINTER(Config)]
    lib.ftg_dgemm_noalloc_max_bytes.argtypes = []
    lib.ftg_workspace_reserve.argtypes = [h, ct.c_size_t]
    lib.ftg_gemm_ex.argtypes = [h, i32, i32, i64, i64, i64, i32, i32, vp, vp, ct.c_float, vp, i64,
                                vp, i64, ct.c_float, vp, i64, vp, ct.POINTER(Config)]
    lib.ftg_dgemm_batched_uneven.argtypes = [h, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                             vp, vp, vp, vp, ct.POINTER(Config)]
    lib.ftg_batched_reserve.argtypes = [h, i64]
    lib.ftg_report_read.argtypes = [h, vp, ct.POINTER(FaultReport), ct.c_int]
    lib.ftg_report_reset.argtypes = [h, vp]
    lib.ftg_last_error_arg.argtypes = [h]
    lib.ftg_tile_info.argtypes = [i32, i32, ct.POINTER(i32), ct.POINTER(i32), ct.POINTER(i32)]
    lib.ftg_tune_set.argtypes = [h, i32, i64, i64, i64, i32]
    lib.ftg_tune_get.argtypes = [h, i32, i64, i64, i64]
    lib.ftg_timing_enable.argtypes = [h, ct.c_int]
    lib.ftg_timing_read.argtypes = [h, ct.POINTER(i32), ct.POINTER(ct.c_double)]
    lib.ftg_status_string.argtypes = [i32]
    lib.ftg_status_string.restype = ct.c_char_p
    for name in EXPORTS:
        if name not in ("ftg_status_string", "ftg_dgemm_noalloc_max_bytes", "ftg_default_lambda"):
            getattr(lib, name).restype = ct.c_int
    lib.ftg_dgemm_noalloc_max_bytes.restype = ct.c_size_t
    lib.ftg_default_lambda.argtypes = []
    lib.ftg_default_lambda.restype = ct.c_double
    _lib = lib
    return lib


def default_lambda() -> float:
    """Threshold scale of the FP32-accumulating paths when the config leaves it 0."""
    return load().ftg_default_lambda()


def tile_info(dtype: int, tile_id: int):
    a, b, c = ct.c_int32(), ct.c_int32(), ct.c_int32()
    st = load().ftg_tile_info(dtype, tile_id, ct.byref(a), ct.byref(b), ct.byref(c))
    return None if st != OK else (a.value, b.value, c.value)


@dataclass
class Report:
    injected: int = 0
    detected: int = 0
    corrected_subtract: int = 0
    corrected_recompute: int = 0
    checksum_only: int = 0
    uncorrectable: int = 0
    tiles_recomputed: int = 0
    lost: int = 0
    max_pass_ratio: float = 0.0
    status: int = OK
    records: list = field(default_factory=list)
    inject_log: list = field(default_factory=list)


def make_config(abft=True, interval_k=0, lam=0.0, correct_policy=0, uncorrectable_policy=0,
                tile=0, seed=None, n_faults=0, per_mac_rate=0.0, bit_lo=0, bit_hi=0,
                target=TARGET_ACC, encode_in_loop=False):
    cfg = Config(int(abft), interval_k, lam, correct_policy, uncorrectable_policy, tile,
                 int(encode_in_loop), None)
    inj = None
    if seed is not None and (n_faults > 0 or per_mac_rate > 0.0):
        inj = Inject(seed & (2**64 - 1), n_faults, target, per_mac_rate, bit_lo, bit_hi)
        cfg.inject = ct.pointer(inj)
    cfg._keep = inj  # keep the injector alive with the config
    return cfg


class Handle:
    """Owns an ftg handle (device report, batched table, tuning table)."""

    def __init__(self, capacity: int = 4096):
        self.lib = load()
        self.h = ct.c_void_p()
        self.capacity = capacity
        st = self.lib.ftg_create(ct.byref(self.h), capacity)
        if st != OK:
            raise FtgError(st, "ftg_create")

    def close(self):
        if self.h:
            self.lib.ftg_destroy(self.h)
            self.h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != OK:
            raise FtgError(st, what, self.lib.ftg_last_error_arg(self.h))

    def dgemm(self, ta, tb, m, n, k, alpha, A_ptr, lda, B_ptr, ldb, beta, C_ptr, ldc,
              stream=None, cfg=None):
        st = self.lib.ftg_dgemm(self.h, ta, tb, m, n, k, alpha, A_ptr, lda, B_ptr, ldb, beta,
                                C_ptr, ldc, stream, ct.byref(cfg) if cfg is not None else None)
        self._check(st, "ftg_dgemm")

    def dgemm_noalloc(self, ta, tb, m, n, k, alpha, A_ptr, lda, B_ptr, ldb, beta, C_ptr, ldc,
                      stream=None, cfg=None):
        st = self.lib.ftg_dgemm_noalloc(self.h, ta, tb, m, n, k, alpha, A_ptr, lda, B_ptr, ldb,
                                        beta, C_ptr, ldc, stream,
                                        ct.byref(cfg) if cfg is not None else None)
        self._check(st, "ftg_dgemm_noalloc")

    def dgemm_unfused(self, ta, tb, m, n, k, alpha, A_ptr, lda, B_ptr, ldb, beta, C_ptr, ldc,
                      stream=None, cfg=None):
        st = self.lib.ftg_dgemm_unfused(self.h, ta, tb, m, n, k, alpha, A_ptr, lda, B_ptr, ldb,
                                        beta, C_ptr, ldc, stream,
                                        ct.byref(cfg) if cfg is not None else None)
        self._check(st, "ftg_dgemm_unfused")

    def dsymm(self, side, uplo, m, n, alpha, A_ptr, lda, B_ptr, ldb, beta, C_ptr, ldc, stream=None,
              cfg=None):
        st = self.lib.ftg_dsymm(self.h, side, uplo, m, n, alpha, A_ptr, lda, B_ptr, ldb, beta, C_ptr,
                                ldc, stream, ct.byref(cfg) if cfg is not None else None)
        self._check(st, "ftg_dsymm")

    def dtrmm(self, side, uplo, ta, diag, m, n, alpha, A_ptr, lda, B_ptr, ldb, stream=None, cfg=None):
        st = self.lib.ftg_dtrmm(self.h, side, uplo, ta, diag, m, n, alpha, A_ptr, lda, B_ptr, ldb,
                                stream, ct.byref(cfg) if cfg is not None else None)
        self._check(st, "ftg_dtrmm")

    def dtrsm(self, side, uplo, ta, diag, m, n, alpha, A_ptr, lda, B_ptr, ldb, stream=None, cfg=None):
        st = self.lib.ftg_dtrsm(self.h, side, uplo, ta, diag, m, n, alpha, A_ptr, lda, B_ptr, ldb,
                                stream, ct.byref(cfg) if cfg is not None else None)
        self._check(st, "ftg_dtrsm")

    def dscal(self, n, alpha, x_ptr, incx, stream=None, cfg=None):
        st = self.lib.ftg_dscal(self.h, n, alpha, x_ptr, incx, stream,
                                ct.byref(cfg) if cfg is not None else None)
        self._check(st, "ftg_dscal")

    def dnrm2(self, n, x_ptr, incx, out_ptr, stream=None, cfg=None):
        st = self.lib.ftg_dnrm2(self.h, n, x_ptr, incx, out_ptr, stream,
                                ct.byref(cfg) if cfg is not None else None)
        self._check(st, "ftg_dnrm2")

    def dgemv(self, ta, m, n, alpha, A_ptr, lda, x_ptr, incx, beta, y_ptr, incy, stream=None, cfg=None):
        st = self.lib.ftg_dgemv(self.h, ta, m, n, alpha, A_ptr, lda, x_ptr, incx, beta, y_ptr, incy,
                                stream, ct.byref(cfg) if cfg is not None else None)
        self._check(st, "ftg_dgemv")

    def dtrsv(self, uplo, ta, diag, n, A_ptr, lda, x_ptr, incx, stream=None, cfg=None):
        st = self.lib.ftg_dtrsv(self.h, uplo, ta, diag, n, A_ptr, lda, x_ptr, incx, stream,
                                ct.byref(cfg) if cfg is not None else None)
        self._check(st, "ftg_dtrsv")

    def workspace_reserve(self, nbytes: int):
        self._check(self.lib.ftg_workspace_reserve(self.h, nbytes), "ftg_workspace_reserve")

    def gemm_ex(self, ta, tb, m, n, k, ab_type, c_type, scale_a, scale_b, alpha, A_ptr, lda,
                B_ptr, ldb, beta, C_ptr, ldc, stream=None, cfg=None):
        st = self.lib.ftg_gemm_ex(self.h, ta, tb, m, n, k, ab_type, c_type, scale_a, scale_b,
                                  alpha, A_ptr, lda, B_ptr, ldb, beta, C_ptr, ldc, stream,
                                  ct.byref(cfg) if cfg is not None else None)
        self._check(st, "ftg_gemm_ex")

    def reset(self, stream=None):
        self._check(self.lib.ftg_report_reset(self.h, stream), "ftg_report_reset")

    def read(self, stream=None) -> Report:
        recs = (FaultRecord * self.capacity)()
        logs = (InjectRecord * self.capacity)()
        out = FaultReport()
        out.capacity = self.capacity
        out.records = ct.cast(recs, ct.POINTER(FaultRecord))
        out.inject_log = ct.cast(logs, ct.POINTER(InjectRecord))
        st = self.lib.ftg_report_read(self.h, stream, ct.byref(out), 1)
        if st not in (OK, ERR_UNCORRECTED):
            raise FtgError(st, "ftg_report_read")
        rep = Report(out.injected, out.detected, out.corrected_subtract, out.corrected_recompute,
                     out.checksum_only, out.uncorrectable, out.tiles_recomputed, out.lost,
                     out.max_pass_ratio, st)
        fields = [f for f, _ in FaultRecord._fields_ if f != "reserved"]
        rep.records = [{f: getattr(r, f) for f in fields}
                       for r in recs[:min(out.n_records, self.capacity)]]
        lf = [f for f, _ in InjectRecord._fields_]
        rep.inject_log = [{f: getattr(r, f) for f in lf}
                          for r in logs[:min(out.n_inject_log, self.capacity)]]
        return rep

    def dgemm_batched(self, plan: "BatchPlan", stream=None, cfg=None, faults_per_problem=None):
        f = None
        if faults_per_problem is not None:
            f = (ct.c_uint32 * plan.count)(*[int(x) for x in faults_per_problem])
        st = self.lib.ftg_dgemm_batched_uneven(
            self.h, plan.count, plan.ta, plan.tb, plan.m, plan.n, plan.k, plan.alpha, plan.A,
            plan.lda, plan.B, plan.ldb, plan.beta, plan.C, plan.ldc, f, stream,
            ct.byref(cfg) if cfg is not None else None)
        self._check(st, "ftg_dgemm_batched_uneven")

    def batched_reserve(self, capacity: int):
        self._check(self.lib.ftg_batched_reserve(self.h, capacity), "ftg_batched_reserve")

    def timing(self, on: bool = True):
        self._check(self.lib.ftg_timing_enable(self.h, int(on)), "ftg_timing_enable")

    def timing_read(self):
        """(launches, total ms) of the product kernels recorded since the last read."""
        n, t = ct.c_int32(), ct.c_double()
        self._check(self.lib.ftg_timing_read(self.h, ct.byref(n), ct.byref(t)), "ftg_timing_read")
        return n.value, t.value

    def tune_set(self, dtype, m, n, k, tile_id):
        self._check(self.lib.ftg_tune_set(self.h, dtype, m, n, k, tile_id), "ftg_tune_set")

    def tune_get(self, dtype, m, n, k) -> int:
        return self.lib.ftg_tune_get(self.h, dtype, m, n, k)


class BatchPlan:
    """Host argument arrays of one batched call (built once, reusable across
    calls and graph captures).  problems: sequence of dicts with keys
    ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc (A/B/C device
    addresses as ints)."""

    def __init__(self, problems):
        cnt = len(problems)
        self.count = cnt
        col = lambda key: [p[key] for p in problems]
        self.ta = (ct.c_int32 * cnt)(*col("ta"))
        self.tb = (ct.c_int32 * cnt)(*col("tb"))
        self.m = (ct.c_int64 * cnt)(*col("m"))
        self.n = (ct.c_int64 * cnt)(*col("n"))
        self.k = (ct.c_int64 * cnt)(*col("k"))
        self.lda = (ct.c_int64 * cnt)(*col("lda"))
        self.ldb = (ct.c_int64 * cnt)(*col("ldb"))
        self.ldc = (ct.c_int64 * cnt)(*col("ldc"))
        self.alpha = (ct.c_double * cnt)(*col("alpha"))
        self.beta = (ct.c_double * cnt)(*col("beta"))
        self.A = (ct.c_void_p * cnt)(*col("A"))
        self.B = (ct.c_void_p * cnt)(*col("B"))
        self.C = (ct.c_void_p * cnt)(*col("C"))


# ---------------------------------------------------------------- torch helpers
def _torch():
    import torch
    return torch


def current_stream_ptr():
    torch = _torch()
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def to_device(a: np.ndarray, dtype=None, device="cuda"):
    """Column-major numpy (rows x cols) -> contiguous torch tensor (cols x rows) on the GPU."""
    torch = _torch()
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(a).T))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device)


def to_host(t) -> np.ndarray:
    """Inverse of to_device: returns a Fortran-ordered (rows x cols) numpy array."""
    return np.asfortranarray(t.detach().cpu().numpy().T)


def ptr(t) -> ct.c_void_p:
    return ct.c_void_p(t.data_ptr())


def gemm_f64(handle: Handle, A, B, C, alpha=1.0, beta=0.0, ta=OP_N, tb=OP_N, cfg=None, m=None,
             n=None, k=None):
    """C := alpha op(A) op(B) + beta C on column-major float64 device tensors (see to_device)."""
    rows_a, cols_a = A.shape[1], A.shape[0]
    rows_b, cols_b = B.shape[1], B.shape[0]
    m = m if m is not None else (cols_a if ta else rows_a)
    k = k if k is not None else (rows_a if ta else cols_a)
    n = n if n is not None else (rows_b if tb else cols_b)
    handle.dgemm(ta, tb, m, n, k, alpha, ptr(A), max(1, rows_a), ptr(B), max(1, rows_b), beta,
                 ptr(C), max(1, C.shape[1]), current_stream_ptr(), cfg)
    return C


def gemm_f64_unfused(handle: Handle, A, B, C, alpha=1.0, beta=0.0, ta=OP_N, tb=OP_N, cfg=None):
    """The unfused comparator (ftg_dgemm_unfused) on column-major float64 device tensors."""
    rows_a, cols_a = A.shape[1], A.shape[0]
    rows_b, cols_b = B.shape[1], B.shape[0]
    m = cols_a if ta else rows_a
    k = rows_a if ta else cols_a
    n = rows_b if tb else cols_b
    handle.dgemm_unfused(ta, tb, m, n, k, alpha, ptr(A), max(1, rows_a), ptr(B), max(1, rows_b),
                         beta, ptr(C), max(1, C.shape[1]), current_stream_ptr(), cfg)
    return C


def dsymm_f64(handle: Handle, A, B, C, alpha=1.0, beta=0.0, side=LEFT, uplo=LOWER, cfg=None):
    """C := alpha A B + beta C (LEFT) or alpha B A + beta C (RIGHT) on column-major
    float64 device tensors; A symmetric, only its `uplo` triangle read."""
    m, n = C.shape[1], C.shape[0]
    handle.dsymm(side, uplo, m, n, alpha, ptr(A), max(1, A.shape[1]), ptr(B), max(1, B.shape[1]), beta,
                 ptr(C), max(1, C.shape[1]), current_stream_ptr(), cfg)
    return C


def dtrmm_f64(handle: Handle, A, B, alpha=1.0, side=LEFT, uplo=LOWER, ta=OP_N, diag=NON_UNIT, cfg=None):
    """B := alpha op(A) B (LEFT) or alpha B op(A) (RIGHT) on column-major float64
    device tensors; A triangular (`uplo` triangle read)."""
    m, n = B.shape[1], B.shape[0]
    handle.dtrmm(side, uplo, ta, diag, m, n, alpha, ptr(A), max(1, A.shape[1]), ptr(B), max(1, B.shape[1]),
                 current_stream_ptr(), cfg)
    return B


def dtrsm_f64(handle: Handle, A, B, alpha=1.0, side=LEFT, uplo=LOWER, ta=OP_N, diag=NON_UNIT, cfg=None):
    """B := alpha op(A)^-1 B (LEFT) or alpha B op(A)^-1 (RIGHT) on column-major
    float64 device tensors; A triangular (`uplo` triangle read)."""
    m, n = B.shape[1], B.shape[0]
    handle.dtrsm(side, uplo, ta, diag, m, n, alpha, ptr(A), max(1, A.shape[1]), ptr(B), max(1, B.shape[1]),
                 current_stream_ptr(), cfg)
    return B


def _vec_len(buf, n, inc):
    if n > 0 and inc != 0 and (n - 1) * abs(inc) >= buf.numel():
        raise FtgError(ERR_INVALID_ARG, "vector buffer shorter than n elements at the stride")


def dscal_f64(handle: Handle, x, alpha, n=None, incx=1, cfg=None):
    """x := alpha x over n elements at stride incx of the float64 device tensor x."""
    n = x.numel() if n is None else n
    _vec_len(x, n, incx)
    handle.dscal(n, alpha, ptr(x), incx, current_stream_ptr(), cfg)
    return x


def dnrm2_f64(handle: Handle, x, out, n=None, incx=1, cfg=None):
    """out[0] := the Euclidean norm of n elements of x at stride incx (out: a
    one-element float64 device tensor)."""
    n = x.numel() if n is None else n
    _vec_len(x, n, incx)
    handle.dnrm2(n, ptr(x), incx, ptr(out), current_stream_ptr(), cfg)
    return out


def dgemv_f64(handle: Handle, A, x, y, alpha=1.0, beta=0.0, ta=OP_N, incx=1, incy=1, cfg=None):
    """y := alpha op(A) x + beta y with A a column-major float64 device tensor
    (see to_device) and x, y 1-D float64 device tensors read at their strides."""
    m, n = A.shape[1], A.shape[0]
    lenx, leny = (m, n) if ta else (n, m)
    _vec_len(x, lenx, incx)
    _vec_len(y, leny, incy)
    handle.dgemv(ta, m, n, alpha, ptr(A), max(1, m), ptr(x), incx, beta, ptr(y), incy,
                 current_stream_ptr(), cfg)
    return y


def dtrsv_f64(handle: Handle, A, x, uplo=LOWER, ta=OP_N, diag=NON_UNIT, incx=1, cfg=None):
    """x := op(A)^-1 x with A a column-major float64 device tensor (the `uplo`
    triangle read) and x a 1-D float64 device tensor read at stride incx."""
    n = A.shape[1]
    _vec_len(x, n, incx)
    handle.dtrsv(uplo, ta, diag, n, ptr(A), max(1, n), ptr(x), incx, current_stream_ptr(), cfg)
    return x


def batch_problem(A, B, C, alpha=1.0, beta=0.0, ta=OP_N, tb=OP_N):
    """One entry of a BatchPlan from column-major device tensors (see to_device)."""
    rows_a, cols_a = A.shape[1], A.shape[0]
    rows_b, cols_b = B.shape[1], B.shape[0]
    return dict(ta=ta, tb=tb, m=cols_a if ta else rows_a, n=rows_b if tb else cols_b,
                k=rows_a if ta else cols_a, alpha=alpha, beta=beta, A=A.data_ptr(),
                lda=max(1, rows_a), B=B.data_ptr(), ldb=max(1, rows_b), C=C.data_ptr(),
                ldc=max(1, C.shape[1]))


def gemm_lowp(handle: Handle, A, B, C, alpha=1.0, beta=0.0, ta=OP_N, tb=OP_N, ab_type=BF16,
              scale_a=None, scale_b=None, cfg=None, m=None, n=None, k=None):
    """C (float32) := alpha s_A s_B op(A) op(B) + beta C on column-major device tensors:
    A, B hold bf16 bit patterns (int16) or e4m3fn codes (uint8); scale_a/scale_b are
    one-element float32 device tensors (FP8 only)."""
    rows_a, cols_a = A.shape[1], A.shape[0]
    rows_b, cols_b = B.shape[1], B.shape[0]
    m = m if m is not None else (cols_a if ta else rows_a)
    k = k if k is not None else (rows_a if ta else cols_a)
    n = n if n is not None else (rows_b if tb else cols_b)
    sa = ptr(scale_a) if scale_a is not None else None
    sb = ptr(scale_b) if scale_b is not None else None
    handle.gemm_ex(ta, tb, m, n, k, ab_type, F32, sa, sb, alpha, ptr(A), max(1, rows_a), ptr(B),
                   max(1, rows_b), beta, ptr(C), max(1, C.shape[1]), current_stream_ptr(), cfg)
    return C
