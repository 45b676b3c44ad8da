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
                     "hp_residuals_workspace_bytes", "hp_residuals", "hp_gemm_sym",
                     "hp_gemm_sym_workspace_bytes"):
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
    assert ctypes.sizeof(hpw.HpResult) == 32 + 7 * 8 + 8 * 8 + 2 * 128 * 8 + 8 + 2 * 8 + 8 + 6 * 8
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
    # autotune scratch: the grouped kinds hold A, B and a table of copies of
    # the result (1 to 64 of them, about 4 Mi outputs in all)
    def tune_bytes(code, M, N, K):
        nb = ctypes.c_size_t()
        rc = lib.hp_autotune_scratch_bytes(code, M, N, K, ctypes.byref(nb))
        return rc, nb.value
    rc, b = tune_bytes(hpw.GEMM_DTYPES["grouped_f64"], 64, 64, 64)
    assert rc == 0 and b >= 8 * (2 * 64 * 64 + 64 * 64 * 64)
    rc, b = tune_bytes(hpw.GEMM_DTYPES["grouped_f32"], 4096, 4096, 64)
    assert rc == 0 and 4 * 4096 * 4096 <= b < 2 * 4 * 4096 * 4096 + (1 << 20)
    assert tune_bytes(8, 64, 64, 64)[0] == EINVAL


EINVAL, EUNSUPPORTED = -1, -5


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
@pytest.mark.parametrize("kw,m,n,code", [
    (dict(chop=-1.0), 10, 10, EINVAL),
    (dict(chop=1e-5, precision="mixed"), 10, 10, EUNSUPPORTED),
    (dict(chop=1e-5, stop="rel_fro_bound"), 10, 10, EUNSUPPORTED),
    (dict(alpha_rule="diag"), 12, 10, EINVAL),
    (dict(method="sm", precision="mixed"), 10, 10, EUNSUPPORTED),
    (dict(kind="drazin", l=2, precision="fp32"), 10, 10, EUNSUPPORTED),
    (dict(kind="drazin", l=2, precision="delta32"), 10, 10, EUNSUPPORTED),
    (dict(method="fm", precision="delta32"), 10, 10, EUNSUPPORTED),
    (dict(chop=1e-5, precision="delta32"), 10, 10, EUNSUPPORTED),
    (dict(device_stop=True, precision="fp32"), 10, 10, EUNSUPPORTED),
    (dict(device_stop=True, stop="rel_fro_bound"), 10, 10, EUNSUPPORTED),
    (dict(device_stop=True, symmetric=True), 10, 10, EUNSUPPORTED),
    (dict(device_stop=True, chop=1e-5), 10, 10, EUNSUPPORTED),
    (dict(kind="drazin", l=2, alpha_rule="norm1inf"), 10, 10, EINVAL),
    (dict(tol=-1.0), 10, 10, EINVAL),
    (dict(max_iter=0), 10, 10, EINVAL),
    (dict(), 0, 10, EINVAL),
    (dict(), 65536, 10, EINVAL),
])
def test_parameter_validation_on_the_host(kw, m, n, code):
    """hp_workspace_bytes runs the same validation as hp_solve, with no GPU."""
    from paper_1604_07893_amd import hyperpower as hpw
    with pytest.raises(hpw.HyperpowerError) as e:
        hpw.workspace_bytes(hpw.make_params(**kw), m, n)
    assert e.value.code == code


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_reserved_fields_must_be_zero():
    from paper_1604_07893_amd import hyperpower as hpw
    p = hpw.make_params()
    p.device_stop = 2  # a flag: 0 or 1
    with pytest.raises(hpw.HyperpowerError):
        hpw.workspace_bytes(p, 10, 10)
    p = hpw.make_params()
    p.reserved[1] = 7
    with pytest.raises(hpw.HyperpowerError):
        hpw.workspace_bytes(p, 10, 10)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_workspace_follows_the_plan():
    """The left form keeps its loop matrices n x n (smaller for m > n); the
    FP32 and 16-bit stages add their own sets; FP32-only keeps one FP64
    iterate."""
    from paper_1604_07893_amd import hyperpower as hpw
    wb = lambda **kw: hpw.workspace_bytes(hpw.make_params(**kw), 4096, 2048)
    left, right = wb(side="left"), wb(side="right")
    assert wb() == left < right
    assert 7 * 4096 * 4096 * 8 < right
    assert wb(precision="fp32") < wb() < wb(precision="fp32_fp64") < wb(precision="mixed")
    assert hpw.workspace_bytes(hpw.make_params(), 8192, 8192) > 10 * 8192 * 8192 * 8


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built (run __graft_entry__.build())")
def test_symmetric_product_argument_checks():
    """hp_gemm_sym / hp_gemm_sym_workspace_bytes reject bad arguments before
    any device work: FP64 and FP32 only, positive sizes, a handle."""
    from paper_1604_07893_amd import hyperpower as hpw
    lib = hpw.load_library()
    nb = ctypes.c_size_t(7)
    assert lib.hp_gemm_sym_workspace_bytes(2, 64, 64, ctypes.byref(nb)) == EINVAL   # 16-bit
    assert lib.hp_gemm_sym_workspace_bytes(0, 0, 64, ctypes.byref(nb)) == EINVAL
    assert lib.hp_gemm_sym_workspace_bytes(1, 64, -1, ctypes.byref(nb)) == EINVAL
    assert lib.hp_gemm_sym_workspace_bytes(0, 64, 64, None) == EINVAL
    # a valid request answers (no device here: nothing to share out, 0 bytes)
    assert lib.hp_gemm_sym_workspace_bytes(0, 2048, 2048, ctypes.byref(nb)) == 0
    assert lib.hp_gemm_sym(None, 0, 64, 64, 1.0, None, 64, None, 64, 0.0, None, 64, None, 0,
                           None) == EINVAL
    # the flag is accepted by the plan of every kind (Drazin simply ignores it)
    for kw in (dict(symmetric=True), dict(symmetric=True, kind="drazin", l=2, alpha_rule="trace")):
        assert hpw.workspace_bytes(hpw.make_params(**kw), 64, 64) > 0
