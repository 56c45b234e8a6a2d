"""Kernel timing hook of the C ABI: event pairs around the product launches."""
import pytest

pytestmark = pytest.mark.gpu


def test_timing_records_product_launches():
    import torch
    from paper_2104_00897_amd import ftgemm
    h = ftgemm.Handle(capacity=64)
    A = torch.rand((512, 512), device="cuda", dtype=torch.float64)
    B = torch.rand((512, 512), device="cuda", dtype=torch.float64)
    C = torch.zeros((512, 512), device="cuda", dtype=torch.float64)
    ftgemm.gemm_f64(h, A, B, C)                    # not recorded: timing off
    h.timing(True)
    for _ in range(3):
        ftgemm.gemm_f64(h, A, B, C)
    n, t = h.timing_read()
    assert n == 3 and t > 0.0
    assert h.timing_read() == (0, 0.0)             # the read clears the record
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):                      # nothing is recorded under capture
        ftgemm.gemm_f64(h, A, B, C)
    g.replay()
    torch.cuda.synchronize()
    assert h.timing_read()[0] == 0
    h.timing(False)
    ftgemm.gemm_f64(h, A, B, C)
    assert h.timing_read()[0] == 0
    del g
    h.close()
