"""Autotuner for the tile-configuration table of the protected GEMM.

The library picks a tile configuration per (operand type, shape bucket) from a
table held by the handle (ftg_tune_set / ftg_tune_get; a bucket is
clamp(ceil(log2 x), 4, 15) of each of m, n and k).  `autotune` times every
candidate configuration of each given shape through the C ABI with HIP events
on the current stream and writes the fastest into the handle; `TuneTable`
keeps the choices and persists them as JSON so a later process can apply them
without re-timing.
"""
from __future__ import annotations

import json
import math

from . import ftgemm

FP64_TILES = (1, 2, 3, 4, 5)
FP64_INTERVAL_TILES = (2, 3, 5)
FP64_BATCHED_TILES = (2, 3)
LOWP_TILES = (1, 2)


def bucket(x: int) -> int:
    """Shape bucket of one dimension (the rule ftg_tune_set applies)."""
    b = 0 if x <= 1 else math.ceil(math.log2(x))
    return min(15, max(4, b))


class TuneTable:
    def __init__(self):
        self.entries: dict[tuple[int, int, int, int], int] = {}

    @staticmethod
    def key(dtype: int, m: int, n: int, k: int):
        return (int(dtype), bucket(m), bucket(n), bucket(k))

    def set(self, dtype, m, n, k, tile_id):
        self.entries[self.key(dtype, m, n, k)] = int(tile_id)

    def get(self, dtype, m, n, k):
        return self.entries.get(self.key(dtype, m, n, k), 0)

    def apply(self, handle) -> None:
        """Writes every entry into the handle (shape = the bucket's upper edge)."""
        for (dt, bm, bn, bk), tile in self.entries.items():
            handle.tune_set(dt, 1 << bm, 1 << bn, 1 << bk, tile)

    def to_json(self) -> str:
        return json.dumps({"version": 1, "entries": [
            {"dtype": k[0], "bm": k[1], "bn": k[2], "bk": k[3], "tile": v}
            for k, v in sorted(self.entries.items())]}, indent=1)

    @classmethod
    def from_json(cls, text: str) -> "TuneTable":
        d = json.loads(text)
        if d.get("version") != 1:
            raise ValueError("unknown tuning-table version")
        t = cls()
        for e in d["entries"]:
            t.entries[(int(e["dtype"]), int(e["bm"]), int(e["bn"]), int(e["bk"]))] = int(e["tile"])
        return t


def _time(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def autotune(handle, shapes, dtype=ftgemm.F64, steps=5, warmup=2, abft=True, interval_k=0,
             table: TuneTable | None = None) -> TuneTable:
    """Times each candidate tile configuration for every (m, n, k) in `shapes`
    (NN, alpha = 1, beta = 0) and records the fastest in `table` and the handle."""
    import torch
    table = table or TuneTable()
    for m, n, k in shapes:
        if dtype == ftgemm.F64:
            cands = FP64_INTERVAL_TILES if interval_k else FP64_TILES
            A = torch.rand((k, m), device="cuda", dtype=torch.float64)
            B = torch.rand((n, k), device="cuda", dtype=torch.float64)
            C = torch.empty((n, m), device="cuda", dtype=torch.float64)

            def run(cfg):
                return ftgemm.gemm_f64(handle, A, B, C, 1.0, 0.0, cfg=cfg)
        else:
            cands = LOWP_TILES
            if dtype == ftgemm.BF16:
                A = torch.rand((k, m), device="cuda").to(torch.bfloat16).view(torch.int16)
                B = torch.rand((n, k), device="cuda").to(torch.bfloat16).view(torch.int16)
                sa = sb = None
            else:
                A = torch.randint(0, 0x78, (k, m), device="cuda", dtype=torch.uint8)
                B = torch.randint(0, 0x78, (n, k), device="cuda", dtype=torch.uint8)
                sa = sb = torch.ones(1, device="cuda")
            C = torch.empty((n, m), device="cuda", dtype=torch.float32)

            def run(cfg):
                return ftgemm.gemm_lowp(handle, A, B, C, 1.0, 0.0, 0, 0, dtype, sa, sb, cfg)
        best, best_ms = 0, float("inf")
        for tile in cands:
            cfg = ftgemm.make_config(abft=abft, interval_k=interval_k, tile=tile)
            ms = _time(torch, lambda: run(cfg), steps, warmup)
            if ms < best_ms:
                best, best_ms = tile, ms
        table.set(dtype, m, n, k, best)
        handle.tune_set(dtype, m, n, k, best)
    return table


def autotune_batched(handle, sizes, steps=3, warmup=1, reps=8, abft=True,
                     table: TuneTable | None = None) -> TuneTable:
    """Tile choice of the batched entry point per shape bucket.  For every bucket
    present in `sizes` ((m, n, k) triples), a batched call of `reps` problems of
    that bucket's first shape (separate outputs, enough tiles to occupy the
    chip as in a mixed batch) is timed with each batched tile configuration,
    and the fastest is recorded in `table` and the handle (a batched call reads
    the handle's table for every problem whose config leaves the tile 0)."""
    import torch
    table = table or TuneTable()
    seen = set()
    stream = ftgemm.current_stream_ptr
    for m, n, k in sizes:
        key = TuneTable.key(ftgemm.F64, m, n, k)
        if key in seen:
            continue
        seen.add(key)
        m, n, k = int(m), int(n), int(k)
        A = torch.rand((k, m), device="cuda", dtype=torch.float64)
        B = torch.rand((n, k), device="cuda", dtype=torch.float64)
        Cs = [torch.empty((n, m), device="cuda", dtype=torch.float64) for _ in range(reps)]
        plan = ftgemm.BatchPlan([ftgemm.batch_problem(A, B, C, 1.0, 0.0) for C in Cs])
        best, best_ms = 0, float("inf")
        for tile in FP64_BATCHED_TILES:
            cfg = ftgemm.make_config(abft=abft, tile=tile)
            ms = _time(torch, lambda: handle.dgemm_batched(plan, stream(), cfg), steps, warmup)
            if ms < best_ms:
                best, best_ms = tile, ms
        table.set(ftgemm.F64, m, n, k, best)
        handle.tune_set(ftgemm.F64, m, n, k, best)
        del A, B, Cs, plan
    return table

