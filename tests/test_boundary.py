"""GPU checks of the C ABI's handle behaviour: report capacity and the repair
queue, workspace growth and its limits (stream capture, captured graphs), the
timing hook across a workspace growth, and the threshold's noise margin.

A full repair queue must never lose a fault silently: the slot is counted and
recorded as uncorrectable, `lost` counts it, and the report read returns
FTG_ERR_UNCORRECTED."""
import numpy as np
import pytest

import oracle
from paper_2104_00897_amd import inputs
from tests.gpu_util import assert_close_f64, magnitude

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2104_00897_amd import ftgemm
    assert torch.cuda.is_available()
    yield ftgemm, torch


def test_small_report_capacity_still_corrects_everything(env):
    """The record capacity only bounds the records kept: 12 faults with room for 4
    records are all corrected, the counters count all of them."""
    ftgemm, torch = env
    h = ftgemm.Handle(capacity=4)
    try:
        m, n, k = 512, 400, 256
        A, B, C = inputs.gemm_operands_f64(m, n, k, seed=21)
        dA, dB, dC = ftgemm.to_device(A), ftgemm.to_device(B), ftgemm.to_device(C)
        h.reset()
        cfg = ftgemm.make_config(tile=3, seed=5, n_faults=12, bit_lo=52, bit_hi=62)
        ftgemm.gemm_f64(h, dA, dB, dC, 1.5, 0.5, cfg=cfg)
        torch.cuda.synchronize()
        rep = h.read()
        assert rep.status == ftgemm.OK and rep.lost == 0
        assert rep.injected == 12 and rep.corrected_subtract + rep.corrected_recompute == 12
        assert len(rep.records) == 4 and len(rep.inject_log) == 4
        ref = oracle.gemm(A, B, C, 1.5, 0.5)
        assert_close_f64(ftgemm.to_host(dC), ref, magnitude(A, B, C, 1.5, 0.5, 0, 0), k)
    finally:
        h.close()


def test_repair_queue_overflow_is_reported(env):
    """More flagged final slots in one call than the repair queue holds (16384):
    64 x 64 tiles over an 8256 x 8192 output give 16512 tiles, each with one
    exponent flip.  The slots that find the queue full are counted uncorrectable
    and `lost`, and the report read returns FTG_ERR_UNCORRECTED; the queued ones
    are corrected."""
    ftgemm, torch = env
    h = ftgemm.Handle(capacity=16)
    try:
        m, n, k = 8256, 8192, 128
        tiles = (m // 64) * (n // 64)
        assert tiles == 16512
        g = torch.Generator(device="cuda").manual_seed(3)
        dA = torch.rand((k, m), generator=g, device="cuda", dtype=torch.float64) * 2 - 1
        dB = torch.rand((n, k), generator=g, device="cuda", dtype=torch.float64) * 2 - 1
        dC = torch.zeros((n, m), device="cuda", dtype=torch.float64)
        cfg = ftgemm.make_config(tile=3, seed=9, n_faults=tiles, bit_lo=56, bit_hi=62)
        h.reset()
        ftgemm.gemm_f64(h, dA, dB, dC, 1.0, 0.0, cfg=cfg)
        torch.cuda.synchronize()
        rep = h.read()
        assert rep.injected == tiles and rep.detected == tiles
        assert rep.lost == tiles - 16384
        assert rep.uncorrectable == rep.lost
        assert rep.corrected_subtract + rep.corrected_recompute == 16384
        assert rep.status == ftgemm.ERR_UNCORRECTED
    finally:
        h.close()


def test_timing_survives_workspace_growth(env):
    """The timing hook keeps working when a later call grows the workspace."""
    ftgemm, torch = env
    h = ftgemm.Handle()
    try:
        h.timing(True)
        for nn in (256, 1024):
            d = torch.rand((nn, nn), device="cuda", dtype=torch.float64)
            c = torch.zeros_like(d)
            ftgemm.gemm_f64(h, d, d, c, 1.0, 0.0)
        launches, ms = h.timing_read()
        h.timing(False)
        assert launches == 2 and ms > 0.0
    finally:
        h.close()


def test_workspace_growth_keeps_captured_buffer(env):
    """A captured graph keeps the workspace's address: a later eager call that
    outgrows the workspace gets a new one while the old one stays allocated,
    so the graph still replays to the eager result (several replays, with
    eager work and synchronisation between them)."""
    ftgemm, torch = env
    h = ftgemm.Handle()
    try:
        nn = 512
        A, B, _ = inputs.gemm_operands_f64(nn, nn, nn, seed=2, with_c=False)
        dA, dB = ftgemm.to_device(A), ftgemm.to_device(B)
        dC = torch.zeros((nn, nn), device="cuda", dtype=torch.float64)
        cfg = ftgemm.make_config(seed=3, n_faults=4, bit_lo=52, bit_hi=62)
        ftgemm.gemm_f64(h, dA, dB, dC, 1.0, 0.0, cfg=cfg)   # eager: sizes the workspace
        torch.cuda.synchronize()
        eager = dC.clone()
        s = torch.cuda.Stream()
        gr = torch.cuda.CUDAGraph()
        dC.zero_()
        with torch.cuda.stream(s):
            with torch.cuda.graph(gr, stream=s):
                ftgemm.gemm_f64(h, dA, dB, dC, 1.0, 0.0, cfg=cfg)
        torch.cuda.synchronize()
        big = torch.rand((2048, 2048), device="cuda", dtype=torch.float64)
        cbig = torch.zeros_like(big)
        ftgemm.gemm_f64(h, big, big, cbig, 1.0, 0.0)      # grows the workspace
        h.workspace_reserve(64 << 20)                       # and again
        torch.cuda.synchronize()
        ref = oracle.gemm(A, B)
        np.testing.assert_allclose(ftgemm.to_host(eager), ref, rtol=0,
                                   atol=1e-12 * nn)
        for _ in range(3):
            dC.zero_()
            gr.replay()
            torch.cuda.synchronize()
            assert torch.equal(dC, eager)
            ftgemm.gemm_f64(h, big, big, cbig, 1.0, 0.0)
            torch.cuda.synchronize()
        del gr
    finally:
        torch.cuda.synchronize()
        h.close()


def test_workspace_reserve_then_calls_fit(env):
    ftgemm, torch = env
    h = ftgemm.Handle()
    try:
        h.workspace_reserve(64 << 20)
        A, B, C = inputs.gemm_operands_f64(700, 600, 500, seed=4)
        dA, dB, dC = ftgemm.to_device(A), ftgemm.to_device(B), ftgemm.to_device(C)
        ftgemm.gemm_f64(h, dA, dB, dC, 1.5, 0.5)
        torch.cuda.synchronize()
        ref = oracle.gemm(A, B, C, 1.5, 0.5)
        assert_close_f64(ftgemm.to_host(dC), ref, magnitude(A, B, C, 1.5, 0.5, 0, 0), 500)
    finally:
        h.close()


def test_noise_margin_reported(env):
    """Fault-free calls report how close rounding came to the threshold: for the
    rigorous FP64 threshold far below 1, never 0 on random data."""
    ftgemm, torch = env
    h = ftgemm.Handle()
    try:
        A, B, C = inputs.gemm_operands_f64(1024, 1024, 1024, seed=6)
        dA, dB, dC = ftgemm.to_device(A), ftgemm.to_device(B), ftgemm.to_device(C)
        h.reset()
        ftgemm.gemm_f64(h, dA, dB, dC, 1.5, 0.5)
        torch.cuda.synchronize()
        rep = h.read()
        assert rep.detected == 0
        assert 0.0 < rep.max_pass_ratio < 0.1
    finally:
        h.close()
