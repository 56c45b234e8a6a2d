"""C ABI library: builds, loads, and exports every symbol include/ftgemm.h declares.

No GPU needed: loading libftgemm.so does not touch the device."""
import ctypes as ct
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ftgemm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ftg_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for want in ["ftg_create", "ftg_destroy", "ftg_dgemm", "ftg_gemm_ex",
                 "ftg_dgemm_batched_uneven", "ftg_report_read", "ftg_report_reset",
                 "ftg_last_error_arg"]:
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2104_00897_amd import ftgemm
    lib = ftgemm.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert missing == []
    assert sorted(ftgemm.EXPORTS) == sorted(declared_functions())


def test_struct_layouts_match_header_sizes():
    from paper_2104_00897_amd import ftgemm
    # fixed-width fields only, natural alignment
    assert ct.sizeof(ftgemm.Inject) == 32
    assert ct.sizeof(ftgemm.Config) == 40
    assert ct.sizeof(ftgemm.FaultRecord) == 56
    assert ct.sizeof(ftgemm.InjectRecord) == 64


def test_status_strings_and_tile_table():
    from paper_2104_00897_amd import ftgemm
    lib = ftgemm.load()
    assert lib.ftg_status_string(0) == b"ok"
    assert lib.ftg_status_string(4) == b"uncorrected fault"
    assert ftgemm.tile_info(ftgemm.F64, 1) == (256, 128, 16)
    assert ftgemm.tile_info(ftgemm.F64, 2) == (128, 128, 16)
    assert ftgemm.tile_info(ftgemm.F64, 3) == (64, 64, 16)
    assert ftgemm.tile_info(ftgemm.F64, 4) == (256, 128, 16)
    assert ftgemm.tile_info(ftgemm.F64, 5) == (128, 128, 16)
    assert ftgemm.tile_info(ftgemm.F64, 9) is None
    # low precision: 128 x 128 checksum tiles; configuration 2 computes 2 x 2 per workgroup
    assert ftgemm.tile_info(ftgemm.BF16, 1) == (128, 128, 64)
    assert ftgemm.tile_info(ftgemm.BF16, 2) == (128, 128, 64)
    assert ftgemm.tile_info(ftgemm.F8_E4M3, 2) == (128, 128, 64)
    assert ftgemm.tile_info(ftgemm.BF16, 3) is None
