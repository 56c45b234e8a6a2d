"""Checksum-protected (ABFT) GEMM for AMD MI355X (gfx950).

The computation runs in hand-written HIP kernels behind the C ABI declared in
include/ftgemm.h; ``ftgemm`` is the ctypes binding, ``inputs`` the seeded
input generators shared by tests and benchmarks.
"""
from . import inputs  # noqa: F401
