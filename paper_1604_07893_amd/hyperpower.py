"""ctypes binding of libhyperpower (the C ABI in include/hyperpower.h).

Argument marshalling only: every step of the iteration runs in the library's
HIP kernels. PyTorch provides device memory (tensors) and the stream; nothing
here computes on the matrices. If the library is missing the calls raise; there
is no fallback.
"""

from __future__ import annotations

import ctypes
import os
import threading
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p

import torch  # loads the HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhyperpower.so")

# ---- constants mirrored from include/hyperpower.h ---------------------------
HP_ABI_VERSION = 4
HP_OK, HP_MAXITER, HP_STAGNATED, HP_DIVERGED, HP_NONFINITE, HP_PENDING = 0, 1, 2, 3, 4, 5
HP_EINVAL, HP_EWORKSPACE, HP_EBUDGET, HP_EHIP, HP_EUNSUPPORTED = -1, -2, -3, -4, -5
STATUS_NAMES = {0: "ok", 1: "maxiter", 2: "stagnated", 3: "diverged", 4: "nonfinite", 5: "pending"}

KIND = {"mp": 0, "moore_penrose": 0, "drazin": 1}
ALPHA = {"norm1inf": 0, "user": 1, "trace": 2, "sigma_max2": 3, "diag": 4}
VARIANT = {"plain": 0, "stabilised": 1, "stabilized": 1, "stab_always": 2}
SIDE = {"auto": 0, "right": 1, "left": 2}
STOP = {"rel_fro": 0, "paper_4_1": 1, "abs_inf": 2, "rel_fro_bound": 3}
METHOD = {"pm": 0, "sm": 1, "cm": 2, "fm": 3, "hm": 4}
METHOD_ORDER = {"pm": 18, "sm": 2, "cm": 3, "fm": 7, "hm": 18}
METHOD_PRODUCTS = {"pm": 7, "sm": 2, "cm": 3, "fm": 5, "hm": 9}
PREC = {"fp64": 0, "fp32": 1, "mixed": 2, "fp32_fp64": 3, "delta32": 4}
LOWP = {"bf16": 0, "f16": 1, "fp16": 1}
FLAG_TIME_KERNELS, FLAG_INF_NORM, FLAG_NO_GRAPH, FLAG_NO_RETRY, FLAG_SYMMETRIC = 1, 2, 4, 8, 16
FLAG_FP64_POLY = 32
DTYPE = {torch.float64: 0, torch.float32: 1}
HP_HIST = 128
NOALLOC_SCRATCH_BYTES = 64 << 20  # HP_NOALLOC_SCRATCH_BYTES


class HpParams(ctypes.Structure):
    _fields_ = [
        ("kind", c_int32), ("drazin_l", c_int32), ("alpha_rule", c_int32), ("variant", c_int32),
        ("alpha", c_double), ("tau_switch", c_double), ("tol", c_double), ("diverge_limit", c_double),
        ("max_iter", c_int32), ("stop_rule", c_int32), ("side", c_int32), ("precision", c_int32),
        ("flags", c_int32), ("low_dtype", c_int32), ("method", c_int32),
        ("device_stop", c_int32), ("chop", c_double), ("reserved", c_int32 * 2),
    ]


class HpResult(ctypes.Structure):
    _fields_ = [
        ("status", c_int32), ("iters", c_int32), ("switch_iter", c_int32), ("side_used", c_int32),
        ("gemms", c_int32), ("iters_stage", c_int32 * 3),
        ("alpha", c_double), ("d_last", c_double), ("stop_last", c_double), ("coc", c_double),
        ("gflop", c_double), ("time_ms", c_double), ("gemm_ms", c_double),
        ("d_stage", c_double * 3), ("gflop_stage", c_double * 3),
        ("queue_ms", c_double), ("run_ms", c_double),
        ("d_hist", c_double * HP_HIST), ("dinf_hist", c_double * HP_HIST),
        ("gemms_sym", c_int32), ("reserved_r", c_int32), ("gflop_sym", c_double),
        ("gemm_ms_sym", c_double),
        ("iters_delta", c_int32), ("reserved_r2", c_int32),
        ("gflop_engine", c_double * 3), ("gemm_ms_engine", c_double * 3),
    ]


class HpProblem(ctypes.Structure):
    _fields_ = [
        ("A", c_void_p), ("m", c_int64), ("n", c_int64), ("lda", c_int64),
        ("X0", c_void_p), ("ldx0", c_int64), ("X", c_void_p), ("ldx", c_int64),
    ]


# Every symbol the header declares, with its ctypes signature.
SIGNATURES = {
    "hp_version": (c_int, []),
    "hp_status_string": (ctypes.c_char_p, [c_int]),
    "hp_params_default": (None, [POINTER(HpParams)]),
    "hp_create": (c_int, [POINTER(c_void_p), c_int]),
    "hp_destroy": (c_int, [c_void_p]),
    "hp_workspace_bytes": (c_int, [POINTER(HpParams), c_int64, c_int64, POINTER(c_size_t)]),
    "hp_complex_workspace_bytes": (c_int, [POINTER(HpParams), c_int64, c_int64, POINTER(c_size_t)]),
    "hp_solve_complex": (c_int, [c_void_p, POINTER(HpParams), c_void_p, c_int64, c_int64, c_int64,
                                 c_void_p, c_int64, c_void_p, c_size_t, c_void_p, POINTER(HpResult)]),
    "hp_solve": (c_int, [c_void_p, POINTER(HpParams), c_void_p, c_int64, c_int64, c_int64,
                         c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_size_t, c_void_p,
                         POINTER(HpResult)]),
    "hp_solve_noalloc": (c_int, [c_void_p, POINTER(HpParams), c_void_p, c_int64, c_int64, c_int64,
                                 c_void_p, c_int64, c_void_p, c_int64, c_void_p,
                                 POINTER(HpResult)]),
    "hp_gemm": (c_int, [c_void_p, c_int, c_int64, c_int64, c_int64, c_double, c_void_p, c_int64,
                        c_void_p, c_int64, c_double, c_void_p, c_int64, c_void_p]),
    "hp_autotune_scratch_bytes": (c_int, [c_int, c_int64, c_int64, c_int64, POINTER(c_size_t)]),
    "hp_gemm_workspace_bytes": (c_int, [c_int, c_int64, c_int64, c_int64, POINTER(c_size_t)]),
    "hp_gemm_sym_workspace_bytes": (c_int, [c_int, c_int64, c_int64, POINTER(c_size_t)]),
    "hp_gemm_sym": (c_int, [c_void_p, c_int, c_int64, c_int64, c_double, c_void_p, c_int64,
                            c_void_p, c_int64, c_double, c_void_p, c_int64, c_void_p, c_size_t,
                            c_void_p]),
    "hp_gemm_ws": (c_int, [c_void_p, c_int, c_int64, c_int64, c_int64, c_double, c_void_p, c_int64,
                           c_void_p, c_int64, c_double, c_void_p, c_int64, c_void_p, c_size_t,
                           c_void_p]),
    "hp_autotune": (c_int, [c_void_p, c_int, c_int64, c_int64, c_int64, c_void_p, c_size_t, c_int,
                            c_void_p, POINTER(c_int), POINTER(c_double)]),
    "hp_tune_export": (c_int, [c_void_p, POINTER(c_int64), c_int, POINTER(c_int)]),
    "hp_tune_import": (c_int, [c_void_p, POINTER(c_int64), c_int]),
    "hp_residuals_workspace_bytes": (c_int, [c_int, c_int, c_int64, c_int64, POINTER(c_size_t)]),
    "hp_residuals": (c_int, [c_void_p, c_int, c_int, c_void_p, c_int64, c_int64, c_int64, c_void_p,
                             c_int64, c_void_p, c_size_t, c_void_p, POINTER(c_double)]),
    "hp_batched_workspace_bytes": (c_int, [POINTER(HpParams), c_int, POINTER(HpProblem),
                                           POINTER(c_size_t)]),
    "hp_solve_batched": (c_int, [c_void_p, POINTER(HpParams), c_int, POINTER(HpProblem), c_void_p,
                                 c_size_t, c_void_p, POINTER(HpResult)]),
    "hp_serve_create": (c_int, [c_void_p, POINTER(HpParams), c_size_t, c_int, c_void_p,
                                POINTER(c_void_p)]),
    "hp_serve_submit": (c_int, [c_void_p, POINTER(HpProblem), POINTER(ctypes.c_uint64)]),
    "hp_serve_step": (c_int, [c_void_p, POINTER(c_int), POINTER(c_int)]),
    "hp_serve_poll": (c_int, [c_void_p, ctypes.c_uint64, POINTER(HpResult)]),
    "hp_serve_destroy": (c_int, [c_void_p]),
}

_lib = None
_lock = threading.Lock()
_handles: dict[int, "Handle"] = {}


def load_library(path: str | None = None) -> ctypes.CDLL:
    """Load libhyperpower.so (built in-tree by __graft_entry__.build())."""
    global _lib
    with _lock:
        if _lib is not None and path is None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise RuntimeError(
                f"libhyperpower.so not found at {p}; build it first "
                "(python -c 'import __graft_entry__ as g; g.build()')")
        lib = ctypes.CDLL(p)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        if lib.hp_version() != HP_ABI_VERSION:
            raise RuntimeError("libhyperpower ABI version mismatch")
        if path is None:
            _lib = lib
        return lib


class HyperpowerError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = load_library()
        super().__init__(f"{where}: {lib.hp_status_string(code).decode()} ({code})")
        self.code = code


class Handle:
    def __init__(self, device: int):
        lib = load_library()
        h = c_void_p()
        rc = lib.hp_create(ctypes.byref(h), device)
        if rc != HP_OK:
            raise HyperpowerError(rc, "hp_create")
        self.ptr = h
        self.device = device

    def __del__(self):
        try:
            if self.ptr:
                load_library().hp_destroy(self.ptr)
        except Exception:
            pass


def handle(device: int | None = None) -> Handle:
    dev = torch.cuda.current_device() if device is None else device
    if dev not in _handles:
        _handles[dev] = Handle(dev)
    return _handles[dev]


def make_params(*, kind="mp", l=0, alpha_rule=None, alpha=0.0, variant="plain", tau_switch=0.1,
                tol=1e-12, max_iter=100, stop="rel_fro", side="auto", precision="fp64",
                diverge_limit=1e6, time_kernels=False, inf_norm=False,
                low_dtype="bf16", graph=True, method="pm", chop=0.0, retry=True,
                symmetric=False, fp64_poly=False, device_stop=False) -> HpParams:
    p = HpParams()
    load_library().hp_params_default(ctypes.byref(p))
    p.kind = KIND[kind]
    p.drazin_l = int(l)
    if alpha_rule is None:
        alpha_rule = "trace" if p.kind == 1 else "norm1inf"
    p.alpha_rule = ALPHA[alpha_rule]
    p.alpha = float(alpha)
    p.variant = VARIANT[variant]
    p.tau_switch = float(tau_switch)
    p.tol = float(tol)
    p.max_iter = int(max_iter)
    p.stop_rule = STOP[stop]
    p.side = SIDE[side]
    p.precision = PREC[precision]
    p.low_dtype = LOWP[low_dtype]
    p.diverge_limit = float(diverge_limit)
    p.method = METHOD[method]
    p.chop = float(chop)
    p.device_stop = 1 if device_stop else 0
    p.flags = ((FLAG_TIME_KERNELS if time_kernels else 0) | (FLAG_INF_NORM if inf_norm else 0)
               | (0 if graph else FLAG_NO_GRAPH) | (0 if retry else FLAG_NO_RETRY)
               | (FLAG_SYMMETRIC if symmetric else 0) | (FLAG_FP64_POLY if fp64_poly else 0))
    return p


def _check_matrix(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a row-major 2-D tensor (stride(1) == 1)")


def workspace_bytes(params: HpParams, m: int, n: int) -> int:
    nb = c_size_t()
    rc = load_library().hp_workspace_bytes(ctypes.byref(params), m, n, ctypes.byref(nb))
    if rc != HP_OK:
        raise HyperpowerError(rc, "hp_workspace_bytes")
    return nb.value


def result_dict(r: HpResult) -> dict:
    it = min(r.iters, HP_HIST)
    return {
        "status": STATUS_NAMES.get(r.status, str(r.status)), "status_code": r.status,
        "iters": r.iters, "switch_iter": r.switch_iter,
        "side": {1: "right", 2: "left"}.get(r.side_used, "?"), "gemms": r.gemms,
        "alpha": r.alpha, "d_last": r.d_last, "stop_last": r.stop_last, "coc": r.coc,
        "gflop": r.gflop, "time_ms": r.time_ms, "gemm_ms": r.gemm_ms,
        "iters_stage": list(r.iters_stage), "d_stage": list(r.d_stage),
        "gflop_stage": list(r.gflop_stage), "queue_ms": r.queue_ms, "run_ms": r.run_ms,
        "d_hist": list(r.d_hist[:it]), "dinf_hist": list(r.dinf_hist[:it]),
        "gemms_sym": r.gemms_sym, "gflop_sym": r.gflop_sym, "gemm_ms_sym": r.gemm_ms_sym,
        "iters_delta": r.iters_delta,
        # by MFMA path: 16-bit operands, FP32, FP64
        "gflop_engine": list(r.gflop_engine), "gemm_ms_engine": list(r.gemm_ms_engine),
    }


def solve(A: torch.Tensor, *, X0: torch.Tensor | None = None, out: torch.Tensor | None = None,
          workspace: torch.Tensor | None = None, stream: torch.cuda.Stream | None = None,
          **kw) -> tuple[torch.Tensor, dict]:
    """Generalized inverse of A (m x n, float64, on the GPU) by the hyperpower
    iteration; returns (X n x m, info). Keyword arguments are those of
    make_params (kind, l, alpha_rule, alpha, variant, tau_switch, tol, max_iter,
    stop, side, ...). Raises HyperpowerError on a negative status; a positive
    status (maxiter/stagnated/diverged/nonfinite) is reported in info."""
    _check_matrix(A, "A")
    m, n = A.shape
    dev = A.device.index if A.device.index is not None else torch.cuda.current_device()
    params = make_params(**kw)
    nbytes = workspace_bytes(params, m, n)
    if workspace is None:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
    if workspace.data_ptr() % 256:
        raise ValueError("workspace must be 256-byte aligned")
    if out is None:
        out = torch.empty((n, m), dtype=torch.float64, device=A.device)
    _check_matrix(out, "out")
    x0p, ldx0 = None, 0
    if X0 is not None:
        _check_matrix(X0, "X0")
        x0p, ldx0 = X0.data_ptr(), X0.stride(0)
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    res = HpResult()
    rc = load_library().hp_solve(
        handle(dev).ptr, ctypes.byref(params), A.data_ptr(), m, n, A.stride(0), x0p, ldx0,
        out.data_ptr(), out.stride(0), workspace.data_ptr(), workspace.numel(), s.cuda_stream,
        ctypes.byref(res))
    if rc < 0:
        raise HyperpowerError(rc, "hp_solve")
    return out, result_dict(res)


def solve_noalloc(A: torch.Tensor, out: torch.Tensor, *, X0: torch.Tensor | None = None,
                  stream: torch.cuda.Stream | None = None, **kw) -> dict:
    """hp_solve_noalloc: as solve(), with the library's fixed device workspace
    (HP_NOALLOC_SCRATCH_BYTES per device) instead of caller memory; the
    caller passes the output `out` (n x m). Returns info."""
    _check_matrix(A, "A")
    _check_matrix(out, "out")
    m, n = A.shape
    if tuple(out.shape) != (n, m):
        raise ValueError("out must be n x m")
    dev = A.device.index if A.device.index is not None else torch.cuda.current_device()
    params = make_params(**kw)
    x0p, ldx0 = None, 0
    if X0 is not None:
        _check_matrix(X0, "X0")
        x0p, ldx0 = X0.data_ptr(), X0.stride(0)
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    res = HpResult()
    rc = load_library().hp_solve_noalloc(
        handle(dev).ptr, ctypes.byref(params), A.data_ptr(), m, n, A.stride(0), x0p, ldx0,
        out.data_ptr(), out.stride(0), s.cuda_stream, ctypes.byref(res))
    if rc < 0:
        raise HyperpowerError(rc, "hp_solve_noalloc")
    return result_dict(res)


def solve_complex(A: torch.Tensor, *, stream: torch.cuda.Stream | None = None,
                  **kw) -> tuple[torch.Tensor, dict]:
    """Generalized inverse of a complex A (m x n, complex128, on the GPU) with
    G = A^* (Moore-Penrose) or A^l (Drazin), through its real 2m x 2n form
    (hp_solve_complex); returns (X n x m complex128, info)."""
    if A.dtype != torch.complex128 or A.dim() != 2 or not A.is_cuda or A.stride(1) != 1:
        raise ValueError("A must be a row-major complex128 CUDA matrix")
    m, n = A.shape
    dev = A.device.index if A.device.index is not None else torch.cuda.current_device()
    params = make_params(**kw)
    lib = load_library()
    nb = c_size_t()
    rc = lib.hp_complex_workspace_bytes(ctypes.byref(params), m, n, ctypes.byref(nb))
    if rc != HP_OK:
        raise HyperpowerError(rc, "hp_complex_workspace_bytes")
    ws = torch.empty(nb.value, dtype=torch.uint8, device=A.device)
    X = torch.empty((n, m), dtype=torch.complex128, device=A.device)
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    res = HpResult()
    rc = lib.hp_solve_complex(handle(dev).ptr, ctypes.byref(params), A.data_ptr(), m, n,
                              A.stride(0), X.data_ptr(), X.stride(0), ws.data_ptr(), ws.numel(),
                              s.cuda_stream, ctypes.byref(res))
    if rc < 0:
        raise HyperpowerError(rc, "hp_solve_complex")
    return X, result_dict(res)


def pinv(A: torch.Tensor, **kw) -> tuple[torch.Tensor, dict]:
    """Moore-Penrose inverse (X0 = alpha A^T, Section 4)."""
    return solve(A, kind="mp", **kw)


def drazin(A: torch.Tensor, l: int, **kw) -> tuple[torch.Tensor, dict]:
    """Drazin inverse with l >= ind(A) (X0 = A^l / Tr(A^{l+1}), Section 4)."""
    return solve(A, kind="drazin", l=l, **kw)


def gemm_workspace_bytes(M: int, N: int, K: int, dtype: str = "f64") -> int:
    """Split-K workspace the default tile choice needs for an M x N x K
    product (0 when it would not split)."""
    nb = c_size_t()
    rc = load_library().hp_gemm_workspace_bytes(GEMM_DTYPES[dtype], M, N, K, ctypes.byref(nb))
    if rc != HP_OK:
        raise HyperpowerError(rc, "hp_gemm_workspace_bytes")
    return nb.value


def gemm(A: torch.Tensor, B: torch.Tensor, *, alpha: float = 1.0, beta_identity: float = 0.0,
         out: torch.Tensor | None = None, stream: torch.cuda.Stream | None = None,
         operands: str | None = None, workspace: torch.Tensor | bool | None = None) -> torch.Tensor:
    """C = alpha A B + beta_identity I on the library's MFMA GEMM kernel.
    operands: None (the tensors' type), or "bf16" / "f16" for float32 tensors
    whose products run on 16-bit MFMA with FP32 accumulation.
    workspace: None (hp_gemm, never split), True (allocate what the default
    tile choice needs and call hp_gemm_ws) or a device uint8 tensor."""
    if A.dtype != B.dtype or A.dtype not in DTYPE:
        raise ValueError("unsupported dtype")
    code = DTYPE[A.dtype]
    if operands is not None:
        if A.dtype != torch.float32:
            raise ValueError("16-bit operands need float32 tensors")
        code = {"bf16": 2, "f16": 3}[operands]
    for t, nm in ((A, "A"), (B, "B")):
        if not t.is_cuda or t.dim() != 2 or t.stride(1) != 1:
            raise ValueError(f"{nm} must be a row-major device matrix")
    M, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    if out is None:
        out = torch.empty((M, N), dtype=A.dtype, device=A.device)
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    dev = A.device.index if A.device.index is not None else torch.cuda.current_device()
    if workspace is None or workspace is False:
        rc = load_library().hp_gemm(handle(dev).ptr, code, M, N, K, alpha, A.data_ptr(),
                                    A.stride(0), B.data_ptr(), B.stride(0), beta_identity,
                                    out.data_ptr(), out.stride(0), s.cuda_stream)
        if rc != HP_OK:
            raise HyperpowerError(rc, "hp_gemm")
        return out
    if workspace is True:
        nb = c_size_t()
        rc = load_library().hp_gemm_workspace_bytes(code, M, N, K, ctypes.byref(nb))
        if rc != HP_OK:
            raise HyperpowerError(rc, "hp_gemm_workspace_bytes")
        workspace = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=A.device)
    rc = load_library().hp_gemm_ws(handle(dev).ptr, code, M, N, K, alpha, A.data_ptr(),
                                   A.stride(0), B.data_ptr(), B.stride(0), beta_identity,
                                   out.data_ptr(), out.stride(0), workspace.data_ptr(),
                                   workspace.numel() * workspace.element_size(), s.cuda_stream)
    if rc != HP_OK:
        raise HyperpowerError(rc, "hp_gemm_ws")
    return out


def gemm_sym(A: torch.Tensor, B: torch.Tensor, *, alpha: float = 1.0, beta_identity: float = 0.0,
             out: torch.Tensor | None = None, stream: torch.cuda.Stream | None = None,
             workspace: torch.Tensor | bool = True) -> torch.Tensor:
    """C = alpha A B + beta_identity I for a product the caller knows to be
    symmetric (hp_gemm_sym): the upper triangle's tiles are computed and
    mirrored. workspace: True (allocate hp_gemm_sym_workspace_bytes), False
    (none: the full product is formed) or a device uint8 tensor."""
    if A.dtype != B.dtype or A.dtype not in DTYPE:
        raise ValueError("unsupported dtype")
    code = DTYPE[A.dtype]
    for t, nm in ((A, "A"), (B, "B")):
        if not t.is_cuda or t.dim() != 2 or t.stride(1) != 1:
            raise ValueError(f"{nm} must be a row-major device matrix")
    N, K = A.shape
    if tuple(B.shape) != (K, N):
        raise ValueError("B must be K x N for an N x K A")
    if out is None:
        out = torch.empty((N, N), dtype=A.dtype, device=A.device)
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    dev = A.device.index if A.device.index is not None else torch.cuda.current_device()
    lib = load_library()
    if workspace is True:
        nb = c_size_t()
        rc = lib.hp_gemm_sym_workspace_bytes(code, N, K, ctypes.byref(nb))
        if rc != HP_OK:
            raise HyperpowerError(rc, "hp_gemm_sym_workspace_bytes")
        workspace = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=A.device)
    if workspace is False:
        ws_ptr, ws_bytes = None, 0
    else:
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    rc = lib.hp_gemm_sym(handle(dev).ptr, code, N, K, alpha, A.data_ptr(), A.stride(0),
                         B.data_ptr(), B.stride(0), beta_identity, out.data_ptr(), out.stride(0),
                         ws_ptr, ws_bytes, s.cuda_stream)
    if rc != HP_OK:
        raise HyperpowerError(rc, "hp_gemm_sym")
    return out


def gemm_bt(A: torch.Tensor, Bt: torch.Tensor, *, alpha: float = 1.0, beta_identity: float = 0.0,
            out: torch.Tensor | None = None, stream: torch.cuda.Stream | None = None) -> torch.Tensor:
    """C = alpha A B + beta_identity I for 16-bit operands held in memory
    (HP_DTYPE_BF16 / HP_DTYPE_F16): A (M x K) and Bt = B^T (N x K), both
    bfloat16 or both float16, row-major with rows of a multiple of 8 elements;
    C is float32 (M x N)."""
    code = {torch.bfloat16: 4, torch.float16: 5}.get(A.dtype)
    if code is None or Bt.dtype != A.dtype:
        raise ValueError("A and Bt must both be bfloat16 or both float16")
    for t, nm in ((A, "A"), (Bt, "Bt")):
        if not t.is_cuda or t.dim() != 2 or t.stride(1) != 1:
            raise ValueError(f"{nm} must be a row-major device matrix")
    M, K = A.shape
    N, K2 = Bt.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    if out is None:
        out = torch.empty((M, N), dtype=torch.float32, device=A.device)
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    dev = A.device.index if A.device.index is not None else torch.cuda.current_device()
    rc = load_library().hp_gemm(handle(dev).ptr, code, M, N, K, alpha, A.data_ptr(), A.stride(0),
                                Bt.data_ptr(), Bt.stride(0), beta_identity, out.data_ptr(),
                                out.stride(0), s.cuda_stream)
    if rc != HP_OK:
        raise HyperpowerError(rc, "hp_gemm")
    return out


def _problem(A: torch.Tensor, X: torch.Tensor, X0: torch.Tensor | None = None) -> HpProblem:
    _check_matrix(A, "A")
    _check_matrix(X, "X")
    m, n = A.shape
    if tuple(X.shape) != (n, m):
        raise ValueError("X must be n x m")
    pr = HpProblem()
    pr.A, pr.m, pr.n, pr.lda = A.data_ptr(), m, n, A.stride(0)
    pr.X, pr.ldx = X.data_ptr(), X.stride(0)
    if X0 is not None:
        _check_matrix(X0, "X0")
        pr.X0, pr.ldx0 = X0.data_ptr(), X0.stride(0)
    return pr


def solve_batched(As: list, *, stream: torch.cuda.Stream | None = None,
                  **kw) -> tuple[list, list]:
    """Generalized inverses of several matrices (uneven shapes) in grouped
    launches; returns ([X_i], [info_i])."""
    if not As:
        return [], []
    dev = As[0].device
    params = make_params(**kw)
    Xs = [torch.empty((a.shape[1], a.shape[0]), dtype=torch.float64, device=dev) for a in As]
    probs = (HpProblem * len(As))(*[_problem(a, x) for a, x in zip(As, Xs)])
    lib = load_library()
    nb = c_size_t()
    rc = lib.hp_batched_workspace_bytes(ctypes.byref(params), len(As), probs, ctypes.byref(nb))
    if rc != HP_OK:
        raise HyperpowerError(rc, "hp_batched_workspace_bytes")
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    outs = (HpResult * len(As))()
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    rc = lib.hp_solve_batched(handle(idx).ptr, ctypes.byref(params), len(As), probs, ws.data_ptr(),
                              ws.numel(), s.cuda_stream, outs)
    if rc != HP_OK:
        raise HyperpowerError(rc, "hp_solve_batched")
    return Xs, [result_dict(o) for o in outs]


class Server:
    """Continuous-batching request server (hp_serve_*): submit() queues a
    request, step() admits what fits the HBM budget and the slot count and runs
    one loop of every admitted request, poll() returns finished results."""

    def __init__(self, *, hbm_budget: int = 1 << 30, max_slots: int = 64,
                 device: int | None = None, stream: torch.cuda.Stream | None = None, **kw):
        self.lib = load_library()
        self.dev = torch.cuda.current_device() if device is None else device
        self.params = make_params(**kw)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.dev)
        ptr = c_void_p()
        rc = self.lib.hp_serve_create(handle(self.dev).ptr, ctypes.byref(self.params),
                                      int(hbm_budget), int(max_slots), self.stream.cuda_stream,
                                      ctypes.byref(ptr))
        if rc != HP_OK:
            raise HyperpowerError(rc, "hp_serve_create")
        self.ptr = ptr
        self._keep: dict[int, tuple] = {}

    def submit(self, A: torch.Tensor, X: torch.Tensor | None = None) -> int:
        if X is None:
            X = torch.empty((A.shape[1], A.shape[0]), dtype=torch.float64, device=A.device)
        pr = _problem(A, X)
        t = ctypes.c_uint64()
        rc = self.lib.hp_serve_submit(self.ptr, ctypes.byref(pr), ctypes.byref(t))
        if rc != HP_OK:
            raise HyperpowerError(rc, "hp_serve_submit")
        self._keep[t.value] = (A, X)  # the library reads A and writes X until done
        return t.value

    def step(self) -> tuple[int, int]:
        a, w = c_int(), c_int()
        rc = self.lib.hp_serve_step(self.ptr, ctypes.byref(a), ctypes.byref(w))
        if rc != HP_OK:
            raise HyperpowerError(rc, "hp_serve_step")
        return a.value, w.value

    def poll(self, ticket: int):
        """None while pending, else (X, info)."""
        r = HpResult()
        rc = self.lib.hp_serve_poll(self.ptr, ticket, ctypes.byref(r))
        if rc == HP_PENDING:
            return None
        if rc < 0:
            raise HyperpowerError(rc, "hp_serve_poll")
        _, X = self._keep.pop(ticket)
        return X, result_dict(r)

    def close(self):
        if getattr(self, "ptr", None):
            self.lib.hp_serve_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


GEMM_DTYPES = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3, "bf16s": 4, "f16s": 5,
               "grouped_f64": 6, "grouped_f32": 7}
GROUPED_TILES = {0: "64x64", 1: "128x128", 2: "32x32 (4x deeper K-tile)"}


def autotune(shapes, dtype: str = "f64", reps: int = 3, device: int | None = None) -> list:
    """Time every tile configuration on each (M, N, K) and keep the fastest in
    the device's handle; returns [(M, N, K, tile, ms)]. With "grouped_f64" or
    "grouped_f32" the grouped launch of batched and served solves is timed on
    a table of copies of the product (ms per product) and groups created
    afterwards use the chosen tile (GROUPED_TILES)."""
    dev = torch.cuda.current_device() if device is None else device
    h = handle(dev)
    code = GEMM_DTYPES[dtype]
    out = []
    for (M, N, K) in shapes:
        nb = c_size_t()
        rc = load_library().hp_autotune_scratch_bytes(code, M, N, K, ctypes.byref(nb))
        if rc != HP_OK:
            raise HyperpowerError(rc, "hp_autotune_scratch_bytes")
        nbytes = nb.value
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{dev}")
        t, ms = c_int(), c_double()
        rc = load_library().hp_autotune(h.ptr, code, M, N, K, scratch.data_ptr(), nbytes, reps,
                                        torch.cuda.current_stream(dev).cuda_stream,
                                        ctypes.byref(t), ctypes.byref(ms))
        if rc != HP_OK:
            raise HyperpowerError(rc, "hp_autotune")
        out.append((M, N, K, t.value, ms.value))
    return out


def tuning_table(device: int | None = None) -> list:
    """The handle's autotuned entries as [(dtype_code, M, N, K, tile)]."""
    dev = torch.cuda.current_device() if device is None else device
    lib, h = load_library(), handle(dev)
    n = c_int()
    lib.hp_tune_export(h.ptr, None, 0, ctypes.byref(n))
    rows = (c_int64 * (5 * max(n.value, 1)))()
    lib.hp_tune_export(h.ptr, rows, n.value, ctypes.byref(n))
    return [tuple(rows[5 * i:5 * i + 5]) for i in range(n.value)]


def save_tuning(path: str, device: int | None = None):
    import json
    with open(path, "w") as f:
        json.dump({"rows": tuning_table(device)}, f)


def load_tuning(path: str, device: int | None = None):
    import json
    with open(path) as f:
        import_tuning(json.load(f)["rows"], device)


def import_tuning(rows, device: int | None = None):
    """Add (dtype_code, M, N, K, tile) rows to the handle's table
    (hp_tune_import); a grouped row also sets the grouped tile of its
    precision for groups created afterwards."""
    dev = torch.cuda.current_device() if device is None else device
    rows = [tuple(int(x) for x in r) for r in rows]
    flat = (c_int64 * (5 * max(len(rows), 1)))(*[x for r in rows for x in r])
    rc = load_library().hp_tune_import(handle(dev).ptr, flat, len(rows))
    if rc != HP_OK:
        raise HyperpowerError(rc, "hp_tune_import")


def residuals(A: torch.Tensor, X: torch.Tensor, kind: str = "mp", l: int = 0) -> list:
    """Relative residuals of the defining equations of X = A^(2), computed on
    the GPU in FP64 (four Penrose equations, or the three Drazin equations)."""
    _check_matrix(A, "A")
    _check_matrix(X, "X")
    m, n = A.shape
    lib = load_library()
    nb = c_size_t()
    rc = lib.hp_residuals_workspace_bytes(KIND[kind], int(l), m, n, ctypes.byref(nb))
    if rc != HP_OK:
        raise HyperpowerError(rc, "hp_residuals_workspace_bytes")
    ws = torch.empty(nb.value, dtype=torch.uint8, device=A.device)
    out = (c_double * 4)()
    dev = A.device.index if A.device.index is not None else torch.cuda.current_device()
    rc = lib.hp_residuals(handle(dev).ptr, KIND[kind], int(l), A.data_ptr(), m, n, A.stride(0),
                          X.data_ptr(), X.stride(0), ws.data_ptr(), ws.numel(),
                          torch.cuda.current_stream(A.device).cuda_stream, out)
    if rc != HP_OK:
        raise HyperpowerError(rc, "hp_residuals")
    return list(out)
