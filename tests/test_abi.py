"""The C-ABI library loads on the CPU and exports every function the public
header declares (no compute calls: there is no GPU here)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hyperpower.h")
LIB = os.path.join(ROOT, "paper_1604_07893_amd", "libhyperpower.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(hp_[a-z_0-9]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hp_version", "hp_status_string", "hp_params_default", "hp_create",
                     "hp_destroy", "hp_workspace_bytes", "hp_solve", "hp_gemm",
                     "hp_batched_workspace_bytes", "hp_solve_batched", "hp_serve_create",
                     "hp_serve_submit", "hp_serve_step", "hp_serve_poll", "hp_serve_destroy",
                     "hp_autotune", "hp_tune_export", "hp_tune_import",
                     "hp_residuals_workspace_bytes", "hp_residuals"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_host_only_calls():
    from paper_1604_07893_amd import hyperpower as hpw
    lib = hpw.load_library()
    assert lib.hp_version() == hpw.HP_ABI_VERSION
    assert lib.hp_status_string(0) == b"ok"
    assert lib.hp_status_string(-2) == b"workspace too small"
    assert set(declared_functions()) == set(hpw.SIGNATURES)
    p = hpw.make_params()
    assert p.tol == 1e-12 and p.max_iter == 100 and abs(p.tau_switch - 0.1) < 1e-15
    # struct layouts mirror the header
    assert ctypes.sizeof(hpw.HpParams) == 96
    assert ctypes.sizeof(hpw.HpResult) == 32 + 7 * 8 + 8 * 8 + 2 * 128 * 8
    assert ctypes.sizeof(hpw.HpProblem) == 8 * 8
    # workspace sizes grow with the problem and reject bad arguments
    small = hpw.workspace_bytes(p, 200, 100)
    big = hpw.workspace_bytes(p, 4096, 2048)
    assert 0 < small < big
    bad = hpw.make_params(kind="drazin", l=3)
    with pytest.raises(hpw.HyperpowerError):
        hpw.workspace_bytes(bad, 10, 12)     # Drazin needs a square matrix
    with pytest.raises(hpw.HyperpowerError):
        hpw.workspace_bytes(hpw.make_params(kind="drazin", l=0), 10, 10)
    with pytest.raises(hpw.HyperpowerError):
        hpw.workspace_bytes(hpw.make_params(alpha_rule="user", alpha=-1.0), 10, 10)
