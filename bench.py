"""Benchmark: generalized inverses per second of the 18th-order hyperpower
iteration on one MI355X, FP64 against the mixed-precision forms.

Headline workload (one step = one complete inverse, inputs resident in HBM):
square nonsingular A = U diag(s) V^T, 8192 x 8192, U and V Haar-orthogonal
(seeded, built on the GPU), s log-uniform in [1e-3, 1] with sigma_max = 1;
X0 = A^T (alpha = 1/sigma_max^2 = 1); plain seven-product loops (Section 2);
every product in FP64; stop at relative Frobenius change < 1e-10. `value` is
its inverses/s.

Beside it in the same JSON line:
  * "mixed_vs_fp64": the same input with 16-bit (bf16) loops, then FP32, then
    FP64 loops (the FP64 stage in the delta form: FP64 residual and update,
    FP32 polynomial), with and without the residual-bound stop, the FP64
    stage with an FP64 polynomial, and FP64 with the bound stop and the
    symmetric products; inverses/s, loops and GFLOP per stage, error against
    the closed form V diag(1/s) U^T, speed-ups over the FP64 value;
  * "roofline": the dominant kernel of the headline (the FP64 MFMA GEMM,
    8192^3 per launch): algorithmic 2*M*N*K flops per launch over its mean
    launch time from hipEvents the library records on the solve stream;
    "roofline_by_dtype": the same for the FP32 and the bf16 GEMM kernels in the
    mixed run, and the bf16 kernel alone at 8192^3;
  * "cpu_baseline": the oracle (numpy FP64) on this host, one loop of the
    same 8192^2 input, scaled to the loops of one FP64 inverse;
  * "extras": the 4096 x 2048 rank-1536 input (stabilised, FP64 / FP32 /
    delta form), a 2048^2 Drazin input, the 200 x 100 latency case, the
    comparison schemes and the Hilbert matrices of Example 8.2, the
    preconditioners of Example 8.3, and the served Poisson stream.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--no-cpu-baseline]
                    [--no-extras] [--extras name,name,...]
    python bench.py --gemm-shapes 8192x8192x8192[,..] [--gemm-dtype f64|f32|bf16|f16|
                    bf16s|f16s|f64sym|f32sym] [--gemm-reps 5] [--check]   # one GEMM kernel alone
    python bench.py --copy-calibration   # a 512 MiB device copy, to scale counters
"""

from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "inverses/s + GEMM TFLOP/s at rel. residual 1e-10, mixed vs FP64; p99 latency"
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}
NSQ, SMIN_SQ, SEED_SQ, TOL = 8192, 1e-3, 1003, 1e-10
WORKLOAD = (f"moore-penrose {NSQ}x{NSQ} square, s log-uniform [{SMIN_SQ:g},1], Haar U/V "
            f"(seed {SEED_SQ}, built on the GPU); X0=A^T (alpha=1/sigma_max^2=1); plain; fp64; "
            f"stop rel. Frobenius change < {TOL:g}")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_gemm_f64_square8192_traffic.json")
GEMM_SRC = os.path.join(ROOT, "paper_1604_07893_amd", "csrc", "hp_gemm.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def trel(torch, a, b):
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


def timed_solves(hpw, torch, A, steps, warmup, **params):
    """Run warmup + steps solves on resident inputs; returns (seconds per
    inverse, infos, X)."""
    dev = A.device
    m, n = A.shape
    nbytes = hpw.workspace_bytes(hpw.make_params(**params), m, n)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    X = torch.empty((n, m), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    for _ in range(warmup):
        hpw.solve(A, out=X, workspace=ws, stream=stream, **params)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(steps):
        _, info = hpw.solve(A, out=X, workspace=ws, stream=stream, **params)
        infos.append(info)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    del ws
    return sec, infos, X


def engine_roofline(infos, engine: int, peak: float, kernel: str) -> dict | None:
    """Executed flops over summed hipEvent time of one MFMA path's launches
    (0: 16-bit operands, 1: FP32, 2: FP64) over the given solves."""
    gf = sum(i["gflop_engine"][engine] for i in infos)
    ms = sum(i["gemm_ms_engine"][engine] for i in infos)
    if gf <= 0 or ms <= 0:
        return None
    a = gf / ms  # GFLOP/ms = TFLOP/s
    return {"bound": "mfma", "kernel": kernel, "achieved": a, "peak": peak, "unit": "TFLOP/s",
            "frac": a / peak, "gflop": gf / len(infos), "gemm_ms": ms / len(infos)}


def measured_traffic():
    """HBM bytes per FP64 GEMM launch from the committed rocprofv3 counter
    summary, if it was taken on the current GEMM source (else None)."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        with open(GEMM_SRC, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None, None
    if rec.get("hp_gemm_hip_sha256") != sha:
        return None, "stale: taken on another hp_gemm.hip"
    return rec["traffic_bytes_per_launch"], os.path.relpath(TRAFFIC_FILE, ROOT)


def blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 0) for i in threadpool_info()
                    if i.get("user_api") == "blas"] or [os.cpu_count()])
    except Exception:  # pragma: no cover
        return os.cpu_count() or 1


def cpu_baseline(A_host: np.ndarray, loops: int) -> dict:
    """The oracle (numpy FP64, OpenBLAS) timed on a bounded sample: one loop
    of (PM) on the full 8192^2 input from X0 = A^T, scaled by the loop count
    of one FP64 inverse."""
    import oracle as O
    X0, _ = O.x0_moore_penrose(A_host, "user", 1.0)
    K = O.pm_constants()
    t0 = time.perf_counter()
    X1 = O.pm_step(A_host, X0, K)
    t_loop = time.perf_counter() - t0
    del X1
    return {"value": 1.0 / (loops * t_loop), "unit": "inverses/s", "cores": int(blas_threads()),
            "kind": "oracle",
            "sample": (f"1 oracle loop of (PM) (7 products, numpy FP64) on the full {NSQ}x{NSQ} "
                       f"input ({t_loop:.1f} s), scaled to the {loops} loops of one FP64 inverse")}


def gemm_standalone(hpw, torch, M, N, K, dtype, reps, check=False, ref_blas=False) -> dict:
    """One GEMM kernel alone: `reps` launches after one warm-up, timed with
    events on the current stream. f64/f32: hp_gemm_ws with a split-K
    workspace; bf16/f16: FP32 operands rounded while staged; bf16s/f16s:
    16-bit operands in memory (A and B^T); f64sym/f32sym: hp_gemm_sym on
    C = G G^T (G random N x K; the symmetric launch forms the upper triangle's
    tiles and mirrors them), algorithmic flops N (N + 1) K."""
    if dtype in ("f64sym", "f32sym"):
        dt = torch.float64 if dtype == "f64sym" else torch.float32
        vec = 2 if dt == torch.float64 else 4
        ldk = -(-K // vec) * vec
        G = torch.randn(N, ldk, dtype=dt, device="cuda")[:, :K]
        Gt = G.t().contiguous()
        C = torch.empty(N, N, dtype=dt, device="cuda")
        nb = ctypes.c_size_t()
        if hpw.load_library().hp_gemm_sym_workspace_bytes(hpw.DTYPE[dt], N, K,
                                                          ctypes.byref(nb)) != 0:
            raise RuntimeError("hp_gemm_sym_workspace_bytes")
        ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device="cuda")
        run = lambda: hpw.gemm_sym(G, Gt, out=C, workspace=ws)
        ref = (lambda: G.double() @ G.double().t()) if check else None
        flops = float(N) * (N + 1) * K
    elif dtype in ("bf16s", "f16s"):
        h = torch.bfloat16 if dtype == "bf16s" else torch.float16
        ldk = -(-K // 8) * 8
        A = torch.randn(M, ldk, device="cuda").to(h)[:, :K]
        Bt = torch.randn(N, ldk, device="cuda").to(h)[:, :K]
        C = torch.empty(M, N, dtype=torch.float32, device="cuda")
        run = lambda: hpw.gemm_bt(A, Bt, out=C)
        ref = (lambda: A.double() @ Bt.double().t()) if check else None
    else:
        dt = torch.float64 if dtype == "f64" else torch.float32
        ops = dtype if dtype in ("bf16", "f16") else None
        vec = 2 if dt == torch.float64 else 4
        lda, ldb = -(-K // vec) * vec, -(-N // vec) * vec
        A = torch.randn(M, lda, dtype=dt, device="cuda")[:, :K]
        B = torch.randn(K, ldb, dtype=dt, device="cuda")[:, :N]
        C = torch.empty(M, N, dtype=dt, device="cuda")
        tiles = -(-M // 128) * -(-N // 128)
        ws = torch.empty(4 * tiles * 128 * 128 * 8 + 4 * 4 * tiles + 4096, dtype=torch.uint8,
                         device="cuda")
        run = lambda: hpw.gemm(A, B, out=C, operands=ops, workspace=ws)
        ref = (lambda: A.double() @ B.double()) if check else None
    if dtype not in ("f64sym", "f32sym"):
        flops = 2.0 * M * N * K
    def timed(fn):
        fn()
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / reps

    ms = timed(run)
    rec = {"dtype": dtype, "M": M, "N": N, "K": K, "ms": ms,
           "tflops": flops / ms * 1e-9}
    if ref_blas:
        # the platform BLAS on the same operands (a reference point, not this
        # library's path): torch.matmul in the operands' dtype
        if dtype in ("bf16s", "f16s"):
            Ac, Bc = A.contiguous(), Bt.t().contiguous()
            blas = lambda: torch.matmul(Ac, Bc)
        elif dtype in ("f64sym", "f32sym"):
            blas = lambda: torch.matmul(G, Gt)
        elif dtype in ("f64", "f32"):
            Ac, Bc = A.contiguous(), B.contiguous()
            blas = lambda: torch.matmul(Ac, Bc)
        else:
            blas = None
        if blas is not None:
            bms = timed(blas)
            rec["torch_matmul_ms"] = bms
            rec["torch_matmul_tflops"] = 2.0 * M * N * K / bms * 1e-9
    if ref is not None:
        R = ref()
        rec["max_rel_err"] = float((C.double() - R).abs().max() / R.abs().max())
    return rec


def copy_calibration(torch):
    """A device copy of known size: a 64 Mi-element FP64 tensor (512 MiB)
    copied three times with torch's copy kernel; each copy reads and writes
    exactly 512 MiB, so the ratio of those bytes to what the FETCH_SIZE /
    WRITE_SIZE counters report per copy scales them for the other kernels."""
    a = torch.empty(64 << 20, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copied_bytes": a.numel() * 8, "copies": 3}), flush=True)


def headline_mixed(hpw, torch, A, closed, steps) -> dict:
    """The 8192^2 input in the mixed-precision forms and the fast FP64 forms."""
    out = {}
    for name, kw in (("mixed", dict(precision="mixed")),
                     ("mixed_bound", dict(precision="mixed", stop="rel_fro_bound")),
                     ("mixed_fp64_poly", dict(precision="mixed", fp64_poly=True)),
                     ("mixed_bound_fp64_poly", dict(precision="mixed", stop="rel_fro_bound",
                                                    fp64_poly=True)),
                     ("fp64_bound", dict(precision="fp64", stop="rel_fro_bound")),
                     ("fp64_bound_sym", dict(precision="fp64", stop="rel_fro_bound",
                                             symmetric=True))):
        sec, infos, X = timed_solves(hpw, torch, A, steps, 1, alpha_rule="user", alpha=1.0,
                                     tol=TOL, time_kernels=True, **kw)
        inf = infos[-1]
        rec = {"inverses_per_s": 1 / sec, "ms_per_inverse": sec * 1e3, "status": inf["status"],
               "iters": inf["iters"], "iters_stage": inf["iters_stage"],
               "iters_delta": inf["iters_delta"],
               "gflop_stage": inf["gflop_stage"], "gflop_per_inverse": inf["gflop"],
               "gflop_by_path": dict(zip(("bf16", "f32", "f64"), inf["gflop_engine"])),
               "gemm_ms_by_path": dict(zip(("bf16", "f32", "f64"), inf["gemm_ms_engine"])),
               "rel_err_vs_closed_form": trel(torch, X, closed)}
        if kw.get("symmetric"):
            rec["sym_launches_per_inverse"] = inf["gemms_sym"]
        if name == "mixed":
            caps = np.cumsum(inf["iters_stage"])
            per_stage = []
            for cap in caps[:2]:
                Xs, _ = hpw.solve(A, alpha_rule="user", alpha=1.0, tol=TOL, precision="mixed",
                                  max_iter=int(cap))
                per_stage.append(trel(torch, Xs, closed))
                del Xs
            per_stage.append(rec["rel_err_vs_closed_form"])
            rec["rel_err_after_stage"] = per_stage
            rec["_infos"] = infos
        out[name] = rec
        del X
        log(f"8192^2 {name}: {1 / sec:.3f} inverses/s, stages {inf['iters_stage']}, "
            f"delta loops {inf['iters_delta']}, err {rec['rel_err_vs_closed_form']:.2e}")
    return out


def extra_lowrank(hpw, torch, steps) -> dict:
    """The rectangular rank-deficient input: 4096 x 2048, rank 1536, s
    log-spaced in [1e-4, 1], Haar U/V (seed 1002); X0 = A^T/sigma_max^2; the
    stabilised variant (switch at relative change < 0.1); tol 1e-10; FP64, all
    FP32, and the delta form (FP64 residual and update, FP32 polynomial)."""
    from paper_1604_07893_amd import inputs
    d = inputs.lowrank_svd(4096, 2048, 1536, smin=1e-4, seed=1002)
    A = torch.from_numpy(d.A).cuda()
    closed = torch.from_numpy((d.V / d.s) @ d.U.T).cuda()
    out = {"workload": "moore-penrose 4096x2048 rank 1536, s log-spaced [1e-4,1], Haar U/V seed "
                       "1002; X0=A^T/sigma_max^2; stabilised; tol 1e-10"}
    for prec in ("fp64", "fp32", "delta32"):
        sec, infos, X = timed_solves(hpw, torch, A, steps, 1, alpha_rule="user", alpha=1.0,
                                     variant="stabilised", tol=TOL, precision=prec,
                                     time_kernels=True)
        inf = infos[-1]
        rec = {"inverses_per_s": 1 / sec, "ms_per_inverse": sec * 1e3, "status": inf["status"],
               "iters": inf["iters"], "switch_iter": inf["switch_iter"], "side": inf["side"],
               "rel_err_vs_closed_form": trel(torch, X, closed)}
        if prec == "fp64":
            rl = engine_roofline(infos, 2, PEAK_TFLOPS["f64"], "FP64 MFMA GEMMs (k_gemm_w4dma from "
                                 "512 output tiles, k_gemm<double> below)")
            rec["gemm_roofline"] = rl
            rec["gflop_per_launch"] = inf["gflop"] / max(inf["gemms"], 1)
        if prec == "fp32":
            rec["note"] = ("every product in FP32: rounding seeds the null-space block, which grows "
                           "18x per plain loop (Theorem 6.2); an FP32 solve switches to the "
                           "stabilised loops (Theorem 7.1) below a change of 0.25 instead of 0.1, "
                           "before that block outgrows X, and ends at its FP32 floor")
            rec["d_hist"] = inf["d_hist"]
        out[prec] = rec
        log(f"4096x2048 {prec}: {rec}")
        del X
    return out


def extra_drazin(hpw, torch, steps):
    from paper_1604_07893_amd import inputs
    d = inputs.drazin_jordan(n=2048, nb=1792, cond_p=10.0, seed=1004)
    nb = d.Q.shape[0]
    J = np.zeros_like(d.A)
    J[:nb, :nb] = (d.Q / d.lam) @ d.Q.T
    closed = d.P @ J @ d.Pinv
    A = torch.from_numpy(d.A).cuda()
    out = {"workload": "drazin 2048x2048, B 1792 (eig U[0.5,2]), nilpotent 256 (index 3), "
                       "cond(P)=10; X0=A^3/Tr(A^4); tol 1e-10"}
    for variant in ("plain", "stabilised"):
        sec, infos, X = timed_solves(hpw, torch, A, steps, 1, kind="drazin", l=3, variant=variant,
                                     tol=TOL)
        out[variant] = {"inverses_per_s": 1 / sec, "status": infos[-1]["status"],
                        "iters": infos[-1]["iters"],
                        "rel_err_vs_closed_form": rel(X.cpu().numpy(), closed)}
    return out


def extra_small(hpw, torch, steps):
    """The 200x100 full-rank case (iid U[-1,1], X0 = A^T/(||A||_1||A||_inf),
    relative Frobenius change < 1e-12): latency-bound; microseconds per
    inverse and the error against the LAPACK pseudo-inverse."""
    from paper_1604_07893_amd import inputs
    A64 = inputs.uniform(200, 100, seed=1001)
    A = torch.from_numpy(A64).cuda()
    ref = np.linalg.pinv(A64)
    out = {"workload": "moore-penrose 200x100, iid U[-1,1] (seed 1001); X0=A^T/(||A||_1||A||_inf); "
                       "stop rel. Frobenius change < 1e-12"}
    sec, infos, X = timed_solves(hpw, torch, A, steps, 3, tol=1e-12)
    out.update({"us_per_inverse": sec * 1e6, "iters": infos[-1]["iters"],
                "status": infos[-1]["status"], "rel_err_vs_lapack_pinv": rel(X.cpu().numpy(), ref)})
    # the stop decisions on the device (hp_params.device_stop): loops enqueued
    # in chunks (a captured graph of two loops replayed), no host read per loop
    sec2, infos2, X2 = timed_solves(hpw, torch, A, steps, 3, tol=1e-12, device_stop=True)
    out["device_stop"] = {"us_per_inverse": sec2 * 1e6, "iters": infos2[-1]["iters"],
                          "status": infos2[-1]["status"],
                          "bitwise_equal_to_host_loop": bool(torch.equal(X2, X))}
    return out


def extra_precond(hpw, torch, steps):
    """Example 8.3's preconditioners on the GPU: X_1 of PM, X_3 of CM and X_5
    of SM from X0 = diag(1/a_ii) (choice3) with Chop[X, 1e-5] after each loop,
    on the seeded 841 x 841 grid-stencil stand-in (the paper's MatrixMarket
    matrix is not available; GMRES and the ILU comparison are not built).
    Reports the time to build each preconditioner, its residual
    ||I - X A||_F / ||I - X0 A||_F and the fraction of nonzero entries."""
    from paper_1604_07893_amd import inputs
    A64 = inputs.grid_stencil()
    A = torch.from_numpy(A64).cuda()
    n = A64.shape[0]
    I = np.eye(n)
    r0 = np.linalg.norm(I - A64 / np.diag(A64)[:, None])
    out = {"workload": "grid stencil 29x29 (841x841, 4089 nonzeros, seed 1006), X0 = diag(1/a_ii), "
                       "Chop[X, 1e-5] after each loop"}
    for mth, loops in (("pm", 1), ("cm", 3), ("sm", 5)):
        sec, infos, X = timed_solves(hpw, torch, A, steps, 3, method=mth, alpha_rule="diag",
                                     max_iter=loops, chop=1e-5)
        Xh = X.cpu().numpy()
        out[f"{mth}_x{loops}"] = {
            "us_per_preconditioner": sec * 1e6, "products": infos[-1]["gemms"],
            "residual_vs_x0": float(np.linalg.norm(I - Xh @ A64) / r0),
            "nonzero_fraction": float(np.count_nonzero(Xh) / Xh.size)}
    return out


def extra_methods(hpw, torch, steps):
    """The comparison of Section 8 on the GPU: every scheme (SM, CM, FM, HM,
    PM) on (a) a square 4096^2 input with kappa = 1e3 (s log-uniform in
    [1e-3, 1], Haar U/V, built on the GPU; X0 = A^T, sigma_max = 1; relative
    Frobenius change < 1e-10) and (b) the Hilbert matrices of Example 8.2,
    H_{m x (m-10)} for m = 100, 200, ..., 1000 (the rows of Tables 2-4) and
    2000, X0 = 2/(sigma_1^2 + sigma_r^2) H^T, rule (stopreliable) with the
    Frobenius norm, eps = 1e-5, 1e-6, 1e-7. sigma_r is read as the smallest
    singular value above sigma_1 * m * 2^-52 (the numerical rank)."""
    from paper_1604_07893_amd import inputs
    order = {"sm": 2, "cm": 3, "fm": 7, "hm": 18, "pm": 18}
    prods = {"sm": 2, "cm": 3, "fm": 5, "hm": 9, "pm": 7}
    out = {"square_4096": {"workload": "square 4096x4096, s log-uniform [1e-3,1], Haar U/V (seed 1006, "
                                       "built on the GPU); X0=A^T; plain FP64; tol 1e-10"}}
    A, U, s, V = inputs.square_svd_device(4096, smin=1e-3, seed=1006)
    closed = (V / s) @ U.T.contiguous()
    for mth in ("sm", "cm", "fm", "hm", "pm"):
        sec, infos, X = timed_solves(hpw, torch, A, steps, 1, method=mth, alpha_rule="user",
                                     alpha=1.0, tol=TOL)
        it = infos[-1]["iters"]
        out["square_4096"][mth] = {
            "inverses_per_s": 1 / sec, "iters": it, "products": infos[-1]["gemms"],
            "efficiency_index": order[mth] ** (1.0 / prods[mth]), "status": infos[-1]["status"],
            "rel_err_vs_closed_form": trel(torch, X, closed)}
    del A, U, s, V, closed
    hil = {"workload": "Hilbert H_{m x (m-10)} (Example 8.2), X0 = 2/(s1^2+sr^2) H^T, rule "
                       "(stopreliable) Frobenius; ms per inverse and loops (the paper's Tables 2-4 "
                       "time the same rows in Mathematica on a 2.4 GHz laptop CPU: context only)"}
    for m in list(range(100, 1001, 100)) + [2000]:
        H = torch.from_numpy(inputs.hilbert(m, m - 10)).cuda()
        sv = torch.linalg.svdvals(H)
        s1 = float(sv[0])
        sr = float(sv[sv > s1 * m * 2.0 ** -52][-1])
        alpha = 2.0 / (s1 * s1 + sr * sr)
        row = {}
        for eps in (1e-5, 1e-6, 1e-7):
            for mth in ("sm", "cm", "hm", "pm"):
                sec, infos, X = timed_solves(hpw, torch, H, steps, 1, method=mth, alpha_rule="user",
                                             alpha=alpha, stop="paper_4_1", tol=eps)
                row[f"{mth}_eps{eps:g}"] = {"ms": sec * 1e3, "iters": infos[-1]["iters"],
                                            "status": infos[-1]["status"]}
        hil[f"H{m}x{m - 10}"] = row
    out["hilbert"] = hil
    return out


def extra_served(hpw, torch, n_req: int, warm: int):
    """Poisson stream of Moore-Penrose requests (m log-uniform in [64, 2048],
    n = m/r, r in {1,2,4}, N(0,1), 10% rank-deficient at half rank) through the
    continuous-batching server, FP32 loops then FP64 (with the Penrose
    projection), at 50/80/95% of the measured saturation rate."""
    from paper_1604_07893_amd import inputs
    kw = dict(variant="stabilised", tol=1e-10, precision="fp32_fp64")
    budget = 32 << 30
    reqs = inputs.request_stream(n_req + warm, qps=1.0, seed=1005)
    mats = [torch.from_numpy(r.A).cuda() for r in reqs]
    torch.cuda.synchronize()

    # accuracy sample after the warm-up: the 6 largest requests and 6 others,
    # against torch's SVD pseudo-inverse on the GPU in FP64 (rank-deficient
    # requests with rcond 1e-10)
    after = list(range(warm, len(reqs)))
    big = sorted(after, key=lambda i: -reqs[i].A.size)[:6]
    rest = [i for i in after if i not in big][:: max(1, len(after) // 6)][:6]
    sample = sorted(set(big + rest))
    kept = {}

    def run(arrivals):
        srv = hpw.Server(hbm_budget=budget, max_slots=64, **kw)
        t0 = time.perf_counter()
        pending = {}
        lat, nxt, done = [], 0, 0
        res = []
        while done < len(mats):
            now = time.perf_counter() - t0
            while nxt < len(mats) and arrivals[nxt] <= now:
                pending[srv.submit(mats[nxt])] = (nxt, arrivals[nxt])
                nxt += 1
            if not pending:
                time.sleep(max(0.0, min(arrivals[nxt] - now, 0.001)))
                continue
            srv.step()
            t_now = time.perf_counter() - t0
            for tk in list(pending):
                r = srv.poll(tk)
                if r is not None:
                    i, arr = pending.pop(tk)
                    lat.append((i, t_now - arr))
                    res.append((i, r[1]))
                    if i in sample or r[1]["status"] != "ok":
                        kept[i] = r[0].clone()
                    done += 1
        wall = time.perf_counter() - t0
        srv.close()
        return wall, lat, res

    pinv_cache = {}

    def pinv_gpu(i):
        if i not in pinv_cache:
            pinv_cache[i] = torch.linalg.pinv(mats[i], rtol=1e-10 if reqs[i].rank_deficient
                                              else 0.0)
        return pinv_cache[i]

    pct = lambda v, q: float(np.percentile(v, q))

    def offered(frac, sat):
        qps = frac * sat
        rng = np.random.default_rng(1005)
        arrivals = np.cumsum(rng.exponential(1.0 / qps, size=len(mats))).tolist()
        wall, lat, res = run(arrivals)
        lat_ms = np.array([l for i, l in sorted(lat) if i >= warm]) * 1e3
        return qps, wall, lat_ms, res

    # the grouped tile: the default (64 x 64) first, then the one hp_autotune
    # picks per precision on the stream's work-weighted median product
    g64, g32 = hpw.GEMM_DTYPES["grouped_f64"], hpw.GEMM_DTYPES["grouped_f32"]
    hpw.import_tuning([(g64, 0, 0, 0, 0), (g32, 0, 0, 0, 0)])
    wall_b, _, _ = run([0.0] * len(mats))
    sat_b = len(mats) / wall_b
    _, _, lat_b, _ = offered(0.8, sat_b)
    dims = sorted(((min(r.A.shape), max(r.A.shape)) for r in reqs),
                  key=lambda d: d[0] * d[0] * d[1])
    w = np.cumsum([d[0] * d[0] * d[1] for d in dims])
    s_med, k_med = dims[int(np.searchsorted(w, w[-1] / 2))]
    tuned = {}
    for name in ("grouped_f64", "grouped_f32"):
        (_, _, _, t, ms), = hpw.autotune([(s_med, s_med, k_med)], dtype=name, reps=5)
        tuned[name] = {"tile": hpw.GROUPED_TILES[t], "us_per_product": ms * 1e3}
    log(f"grouped tile before: saturation {sat_b:.0f}/s p99@80% {pct(lat_b, 99):.1f} ms; "
        f"autotuned on {s_med}x{s_med}x{k_med}: {tuned}")

    # saturation: everything arrives at t = 0
    wall0, _, res0 = run([0.0] * len(mats))
    sat = len(mats) / wall0
    gflop_all = sum(r["gflop"] for _, r in res0)
    served_err = {i: trel(torch, kept[i], pinv_gpu(i)) for i in sample}
    not_ok = {i: (r["status"], trel(torch, kept[i], pinv_gpu(i)), reqs[i].A.shape,
                  reqs[i].rank_deficient)
              for i, r in res0 if r["status"] != "ok"}
    # the plain FP64 GPU method on the same requests, one hp_solve after another
    kw64 = dict(variant="stabilised", tol=1e-10, precision="fp64")
    for A in mats[:warm]:
        hpw.solve(A, **kw64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    seq_status, seq_err = [], []
    for i, A in enumerate(mats):
        X, info = hpw.solve(A, **kw64)
        seq_status.append(info["status"])
        if i in sample:
            seq_err.append(trel(torch, X, pinv_gpu(i)))
    torch.cuda.synchronize()
    seq_rate = len(mats) / (time.perf_counter() - t0)
    out = {"workload": (f"{n_req} Poisson requests (+{warm} warm-up), m log-uniform [64,2048], "
                        "n=m/r r in {1,2,4}, N(0,1), 10% rank-deficient; FP32 loops + FP64 "
                        "final loops in grouped launches; budget 32 GiB, 64 slots; offered at "
                        "50/80/95% of the saturation rate (headline: 80%)"),
           "saturation_req_per_s": sat,
           "executed_tflops_at_saturation": gflop_all / wall0 * 1e-3,
           "plain_fp64_sequential": {
               "what": "the same requests solved one after another by hp_solve, FP64, stabilised, "
                       "tol 1e-10 (the plain FP64 GPU method)",
               "inverses_per_s": seq_rate,
               "ok_fraction": seq_status.count("ok") / len(seq_status),
               "rel_err_vs_pinv_max_sample": max(seq_err)},
           "served_rel_err_vs_pinv_max_sample": max(served_err.values()),
           "served_rel_err_vs_pinv_largest": {
               f"{reqs[i].A.shape[0]}x{reqs[i].A.shape[1]}": served_err[i] for i in big},
           "served_not_ok": [{"status": v[0], "rel_err_vs_pinv": v[1], "shape": list(v[2]),
                              "rank_deficient": bool(v[3])} for v in not_ok.values()],
           "accuracy_sample": (f"{len(sample)} requests after the warm-up (the 6 largest and "
                               "6 spread over the trace), relative Frobenius error against "
                               "torch.linalg.pinv (SVD, FP64, on the GPU)"),
           "speedup_saturation_vs_plain_fp64": sat / seq_rate}
    for frac in (0.5, 0.8, 0.95):
        qps, wall, lat_ms, res = offered(frac, sat)
        rd = dict(res)
        q_ms = np.array([rd[i]["queue_ms"] for i in sorted(rd) if i >= warm])
        r_ms = np.array([rd[i]["run_ms"] for i in sorted(rd) if i >= warm])
        statuses = [r["status"] for i, r in res]
        rec = {"offered_qps": qps, "inverses_per_s": len(mats) / wall,
               "p50_ms": pct(lat_ms, 50), "p99_ms": pct(lat_ms, 99),
               "queue_p50_ms": pct(q_ms, 50), "queue_p99_ms": pct(q_ms, 99),
               "run_p50_ms": pct(r_ms, 50), "run_p99_ms": pct(r_ms, 99),
               "ok_fraction": statuses.count("ok") / len(statuses),
               "status_counts": {k: statuses.count(k) for k in sorted(set(statuses))}}
        out[f"at_{int(frac * 100)}pct"] = rec
        log(f"served at {int(frac * 100)}%: {rec}")
        if frac == 0.8:
            out.update({k: rec[k] for k in ("offered_qps", "inverses_per_s", "p50_ms", "p99_ms",
                                            "ok_fraction")})
    out["grouped_tile"] = {
        "what": ("tile of the grouped launches: the default 64x64 (before) and the one "
                 "hp_autotune picks per precision on the stream's work-weighted median "
                 f"product {s_med}x{s_med}x{k_med} (after; the rest of this record)"),
        "autotuned": tuned,
        "before": {"tile": "64x64", "saturation_req_per_s": sat_b,
                   "p99_ms_at_80pct": pct(lat_b, 99)},
        "after": {"saturation_req_per_s": sat, "p99_ms_at_80pct": out.get("p99_ms")}}
    hpw.import_tuning([(g64, 0, 0, 0, 0), (g32, 0, 0, 0, 0)])
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision forms")
    ap.add_argument("--extras", default="",
                    help="comma-separated names of the extras to run (default: all)")
    ap.add_argument("--gemm-shapes", default="", help="MxNxK list: time one GEMM kernel alone")
    ap.add_argument("--gemm-dtype", default="f64",
                    choices=["f64", "f32", "bf16", "f16", "bf16s", "f16s", "f64sym", "f32sym"])
    ap.add_argument("--gemm-reps", type=int, default=5)
    ap.add_argument("--check", action="store_true", help="--gemm-shapes: compare with torch FP64")
    ap.add_argument("--gemm-ref", action="store_true",
                    help="--gemm-shapes: also time torch.matmul (the platform's BLAS) on the same "
                         "operands and dtype, for reference only")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--host-input", action="store_true",
                    help="build the 8192^2 input with numpy on the host (same recipe, other "
                         "draws): torch's GPU QR does not run under rocprofv3 counter collection")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the hyperpower "
              "solver here has no multi-GPU path.", file=sys.stderr)
        return 2

    import torch
    from paper_1604_07893_amd import hyperpower as hpw
    from paper_1604_07893_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        copy_calibration(torch)
        return 0
    if args.gemm_shapes:
        for spec in args.gemm_shapes.split(","):
            M, N, K = (int(v) for v in spec.lower().split("x"))
            print(json.dumps(gemm_standalone(hpw, torch, M, N, K, args.gemm_dtype, args.gemm_reps,
                                             args.check, args.gemm_ref)), flush=True)
        return 0

    if args.host_input:
        d = inputs.square_svd(NSQ, smin=SMIN_SQ, seed=SEED_SQ)
        A = torch.from_numpy(d.A).cuda()
        closed = torch.from_numpy((d.V / d.s) @ d.U.T).cuda()
        del d
    else:
        A, U, s, V = inputs.square_svd_device(NSQ, smin=SMIN_SQ, seed=SEED_SQ)
        closed = (V / s) @ U.T.contiguous()  # V diag(1/s) U^T: a reference, not the method
        del U, V, s
    torch.cuda.synchronize()
    params = dict(alpha_rule="user", alpha=1.0, tol=TOL, precision="fp64")
    sec, infos, X = timed_solves(hpw, torch, A, args.steps, args.warmup, time_kernels=True,
                                 **params)
    err = trel(torch, X, closed)
    del X
    last = infos[-1]
    launches = sum(i["gemms"] for i in infos)
    rl = engine_roofline(infos, 2, PEAK_TFLOPS["f64"],
                         "k_gemm_w4dma (FP64 MFMA GEMM, 4 waves of 64x64, load-to-LDS tiles, "
                         f"with the fused loop epilogue), {NSQ}x{NSQ}x{NSQ} per launch")
    traffic, traffic_src = measured_traffic()
    roofline = {
        "bound": "mfma", "kernel": rl["kernel"], "achieved": rl["achieved"],
        "peak": PEAK_TFLOPS["f64"], "unit": "TFLOP/s", "frac": rl["frac"],
        "traffic": traffic,
        "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        "traffic_source": traffic_src,
        "gflop_per_launch": sum(i["gflop"] for i in infos) / max(launches, 1),
        "avg_launch_ms": sum(i["gemm_ms"] for i in infos) / max(launches, 1),
        "timing": "hipEvents recorded by the library around each GEMM launch on the solve "
                  "stream, over the timed steps",
    }
    line = {
        "metric": METRIC,
        "value": 1.0 / sec,
        "unit": "inverses/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD + (" (built on the host)" if args.host_input else ""),
                   "m": NSQ, "n": NSQ, "smin": SMIN_SQ, "variant": "plain",
                   "precision": "fp64", "tol": TOL},
        "roofline": roofline,
        "iters": last["iters"],
        "status": last["status"],
        "rel_err_vs_closed_form": err,
        "gemm_tflops_executed": last["gflop"] / (sec * 1e3),
    }
    log(f"headline: {1 / sec:.3f} inverses/s ({sec * 1e3:.1f} ms), {last['iters']} loops, "
        f"FP64 GEMM {rl['achieved']:.1f} TFLOP/s, err {err:.2e}")
    if not args.no_mixed:
        mx = headline_mixed(hpw, torch, A, closed, 2)
        minf = mx["mixed"].pop("_infos")
        fp64_rate = 1.0 / sec
        for k in list(mx):
            mx[k]["speedup_vs_fp64"] = mx[k]["inverses_per_s"] / fp64_rate
        line["mixed_vs_fp64"] = mx
        bd = {"f64": {k: v for k, v in roofline.items() if k not in ("traffic", "traffic_unit",
                                                                      "traffic_source", "timing")}}
        bd["f32"] = engine_roofline(minf, 1, PEAK_TFLOPS["f32"],
                                    "k_gemm_w4dma_f32 (FP32 MFMA, 4 waves of 128x128 per 256x256 tile, "
                                    "load-to-LDS), mixed run: FP32 stage and the "
                                    "delta-form polynomials of the FP64 stage, 8192^3")
        bd["bf16"] = engine_roofline(minf, 0, PEAK_TFLOPS["bf16"],
                                     "k_gemm_h16_dma (bf16 operands, FP32 accumulate), mixed run's "
                                     "16-bit stage, 8192^3")
        alone = gemm_standalone(hpw, torch, NSQ, NSQ, NSQ, "bf16s", 5)
        bd["bf16_alone"] = {"bound": "mfma", "kernel": "k_gemm_h16_dma alone, 8192^3",
                            "achieved": alone["tflops"], "peak": PEAK_TFLOPS["bf16"],
                            "unit": "TFLOP/s", "frac": alone["tflops"] / PEAK_TFLOPS["bf16"]}
        line["roofline_by_dtype"] = bd
    if not args.no_cpu_baseline:
        A_host = A.cpu().numpy()
        line["cpu_baseline"] = cpu_baseline(A_host, last["iters"])
        del A_host
    del A, closed
    torch.cuda.empty_cache()
    if not args.no_extras:
        extras = {}
        for name, fn in (("lowrank_4096x2048", lambda: extra_lowrank(hpw, torch, 5)),
                         ("drazin_2048", lambda: extra_drazin(hpw, torch, 3)),
                         ("small_200x100", lambda: extra_small(hpw, torch, 50)),
                         ("methods", lambda: extra_methods(hpw, torch, 2)),
                         ("preconditioner_example_8_3", lambda: extra_precond(hpw, torch, 20)),
                         ("served_stream", lambda: extra_served(hpw, torch, 2000, 200))):
            if args.extras and name not in args.extras.split(","):
                continue
            t0 = time.perf_counter()
            try:
                extras[name] = fn()
            except Exception as e:  # a failing extra must not hide the headline
                extras[name] = {"error": f"{type(e).__name__}: {e}"}
            torch.cuda.empty_cache()
            log(f"extra {name} done in {time.perf_counter() - t0:.1f} s")
        line["extras"] = extras
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
