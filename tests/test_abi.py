"""The C-ABI library loads on the host and exports every entry point that
include/bamg.h declares (no GPU work is issued)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "bamg.h")
LIB = os.path.join(ROOT, "paper_1308_5992_amd", "libbamg.so")


def declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bamg_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ["bamg_setup", "bamg_solve", "bamg_solve_batch", "bamg_apply_dhat", "bamg_free",
                 "bamg_export_level", "bamg_import_level", "bamg_footprint_bytes", "bamg_last_error",
                 "bamg_default_params"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libbamg.so not built")
    lib = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(lib, name), name


def test_host_only_entry_points():
    """default params and the footprint query run on the host."""
    if not os.path.exists(LIB):
        pytest.skip("libbamg.so not built")
    import paper_1308_5992_amd as b
    p = b.bamg_default_params(N=256)
    assert (p.max_coarse, p.n_tv, p.pre, p.post, p.restart) == (8192, 8, 4, 4, 32)
    fb = b.bamg_footprint_bytes(p)
    assert 50 * 2 ** 20 < fb < 2 * 2 ** 30
    assert b.bamg_footprint_bytes(b.bamg_default_params(N=36)) == 0
    assert b.bamg_footprint_bytes(b.bamg_default_params(N=512)) > fb
    # the FP32 copies of the 8192 x 8192 coarsest inverse, mixed precisions only: the whole
    # matrix (8 n^2 bytes) and its packed 64 x 64 blocks on and above the diagonal
    # (8 (n^2 / 2 + 32 n) bytes)
    assert p.coarsest_fp32 == 0
    n = 8192
    f16 = b.bamg_footprint_bytes(b.bamg_default_params(N=256, precision=1))
    f16c = b.bamg_footprint_bytes(b.bamg_default_params(N=256, precision=1, coarsest_fp32=1))
    assert f16c - f16 == 8 * n ** 2 + 8 * (n ** 2 // 2 + 32 * n)
    assert b.bamg_footprint_bytes(b.bamg_default_params(N=256, coarsest_fp32=1)) == 0
    # look-ahead of the single-RHS FGMRES: on by default, 0 / 1 / 2 valid, other values rejected
    assert p.lookahead == 1
    for la in (0, 2):
        assert b.bamg_footprint_bytes(b.bamg_default_params(N=256, lookahead=la)) == fb
    assert b.bamg_footprint_bytes(b.bamg_default_params(N=256, lookahead=3)) == 0
    assert b.bamg_footprint_bytes(b.bamg_default_params(N=256, lookahead=-1)) == 0
