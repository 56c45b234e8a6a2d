"""Seeded synthetic inputs shared by the GPU path's tests/benchmarks and the CPU oracle.

This module holds none of the method's arithmetic: it only draws random
operands (numpy PCG64 streams) and rounds them to the operand dtypes.  The
paper measures square random matrices of 2048^2..10240^2 (§6); the shapes
used here are the benchmark workloads (FP64 8192^3, bf16/fp8 8192^3, a
transformer-sized linear layer, 512 log-uniform batched problems) and small
ragged cases for the tests.

All matrices are returned as numpy arrays in Fortran (column-major) order,
as the BLAS-style interface expects.
"""
from __future__ import annotations

import numpy as np


def uniform_f64(rng: np.random.Generator, rows: int, cols: int, lo=-1.0, hi=1.0) -> np.ndarray:
    return np.asfortranarray(rng.uniform(lo, hi, size=(cols, rows)).T)


def gemm_operands_f64(m, n, k, seed=0, ta=0, tb=0, with_c=True, lo=-1.0, hi=1.0):
    """A, then B, then C drawn i.i.d. U[lo, hi] from one PCG64 stream.

    Stored shapes follow the transpose flags: A is (m,k) for ta=0 and (k,m)
    for ta=1; B is (k,n) for tb=0 and (n,k) for tb=1; C is (m,n)."""
    rng = np.random.default_rng(seed)
    A = uniform_f64(rng, *((k, m) if ta else (m, k)), lo, hi)
    B = uniform_f64(rng, *((n, k) if tb else (k, n)), lo, hi)
    C = uniform_f64(rng, m, n, lo, hi) if with_c else None
    return A, B, C


def integer_operands(m, n, k, seed=0, ta=0, tb=0, lo=-8, hi=8):
    """Small-integer operands: every product and partial sum is exact in binary64
    (and in binary32 while k*max|a||b| < 2^24), so checksum identities hold bitwise."""
    rng = np.random.default_rng(seed)
    shp_a = (k, m) if ta else (m, k)
    shp_b = (n, k) if tb else (k, n)
    A = np.asfortranarray(rng.integers(lo, hi + 1, size=shp_a).astype(np.float64))
    B = np.asfortranarray(rng.integers(lo, hi + 1, size=shp_b).astype(np.float64))
    C = np.asfortranarray(rng.integers(lo, hi + 1, size=(m, n)).astype(np.float64))
    return A, B, C


def log_uniform_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """(count, 3) array of m, n, k, each round(exp(U(ln lo, ln hi))) clipped to [lo, hi]."""
    rng = np.random.default_rng(seed)
    x = np.exp(rng.uniform(np.log(lo), np.log(hi), size=(count, 3)))
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


def normal_f32(rng: np.random.Generator, rows: int, cols: int, std=1.0) -> np.ndarray:
    return np.asfortranarray(rng.standard_normal(size=(cols, rows)).T.astype(np.float32) * std)


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even binary32 -> bfloat16; returns the uint16 bit patterns."""
    x = np.asarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)
    return r


def bf16_bits_to_f64(b: np.ndarray) -> np.ndarray:
    u = (b.astype(np.uint32) << 16)
    return u.view(np.float32).astype(np.float64)


def e4m3_table() -> np.ndarray:
    """The 256 OCP float8 e4m3fn values (NaN for the two NaN codes), from the format's definition:
    1 sign bit, 4 exponent bits (bias 7), 3 mantissa bits, no infinities, S.1111.111 = NaN."""
    vals = np.empty(256)
    for code in range(256):
        s = -1.0 if code & 0x80 else 1.0
        e = (code >> 3) & 0xF
        f = code & 0x7
        if e == 0xF and f == 0x7:
            vals[code] = np.nan
        elif e == 0:
            vals[code] = s * (f / 8.0) * 2.0 ** (-6)
        else:
            vals[code] = s * (1.0 + f / 8.0) * 2.0 ** (e - 7)
    return vals


def to_e4m3_bits(x: np.ndarray) -> np.ndarray:
    """Saturating round-to-nearest-even binary64 -> e4m3fn codes (uint8)."""
    tab = e4m3_table()
    finite = np.where(np.isnan(tab), np.inf, tab)
    pos_codes = np.arange(0, 0x7F)           # 0x00..0x7E, ascending values
    pos_vals = finite[pos_codes]
    a = np.clip(np.abs(np.asarray(x, dtype=np.float64)), 0.0, 448.0)
    idx = np.searchsorted(pos_vals, a)        # first value >= a
    idx = np.clip(idx, 0, len(pos_vals) - 1)
    lo_idx = np.clip(idx - 1, 0, len(pos_vals) - 1)
    hi_v = pos_vals[idx]
    lo_v = pos_vals[lo_idx]
    d_hi = hi_v - a
    d_lo = a - lo_v
    pick_hi = (d_hi < d_lo) | ((d_hi == d_lo) & ((pos_codes[idx] & 1) == 0))
    code = np.where(pick_hi, pos_codes[idx], pos_codes[lo_idx]).astype(np.uint8)
    neg = np.signbit(np.asarray(x, dtype=np.float64)) & (code != 0)
    return np.where(neg, code | 0x80, code).astype(np.uint8)


def quantize_e4m3(x: np.ndarray):
    """Per-tensor absmax scaling: s = absmax(x)/448 (binary32), q = RNE_e4m3fn(x/s).
    Returns (codes uint8 in x's layout, s as float32)."""
    amax = float(np.max(np.abs(x))) if x.size else 0.0
    s = np.float32(amax / 448.0) if amax > 0 else np.float32(1.0)
    q = to_e4m3_bits(np.asarray(x, dtype=np.float64) / np.float64(s))
    return q, s
