"""Benchmark: Moore-Penrose inverses per second of the 18th-order hyperpower
iteration on one MI355X.

Workload (one step = one complete inverse, inputs resident in HBM):
rectangular rank-deficient A = U diag(s) V^T, 4096 x 2048, rank 1536, U and V
Haar-orthogonal (seeded), nonzero s log-spaced in [1e-4, 1]; X0 = A^T /
sigma_max^2 (sigma_max = 1 by construction); the stabilised variant (plain
seven-product loops, then X <- X A X loops once the relative change drops below
0.1); FP64; stop at relative Frobenius change < 1e-10.

Prints one JSON line with the throughput, the roofline of the dominant kernel
(the FP64 MFMA GEMM: executed 2MNK flops over its summed hipEvent time on the
solve stream) and a CPU baseline (the oracle timed on this host).

    python bench.py [--gpus 1] [--steps 10] [--warmup 2] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "inverses/s + GEMM TFLOP/s at rel. residual 1e-10, mixed vs FP64; p99 latency"
PEAK_FP64_TFLOPS = 78.6
M, N, RANK, SMIN, SEED, TOL = 4096, 2048, 1536, 1e-4, 1002, 1e-10
WORKLOAD = (f"moore-penrose {M}x{N} rank {RANK}, s log-spaced [{SMIN:g},1], Haar U/V seed {SEED}; "
            f"X0=A^T/sigma_max^2; stabilised (switch at rel. change < 0.1); fp64; "
            f"stop rel. Frobenius change < {TOL:g}")


def cpu_baseline(d, n_plain: int, n_stab: int) -> dict:
    """The oracle (numpy FP64, OpenBLAS) timed on a bounded sample: one plain
    and one stabilised loop on the full-size input, scaled by the loop counts
    of a full inverse."""
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 0) for i in threadpool_info()
                     if i.get("user_api") == "blas"] or [os.cpu_count()])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    A = d.A
    X0, _ = O.x0_moore_penrose(A, "user", 1.0)
    K = O.pm_constants()
    t0 = time.perf_counter()
    X1 = O.pm_step(A, X0, K)
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    X2 = O.stabilise(A, O.pm_step(A, X1, K))
    t_stab = time.perf_counter() - t0
    del X2
    t_inv = n_plain * t_plain + n_stab * t_stab
    return {"value": 1.0 / t_inv, "unit": "inverses/s", "cores": int(cores), "kind": "oracle",
            "sample": (f"1 plain + 1 stabilised oracle loop on the full {M}x{N} input "
                       f"({t_plain:.2f} s + {t_stab:.2f} s), scaled to {n_plain} plain + "
                       f"{n_stab} stabilised loops per inverse")}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the hyperpower "
              "solver here has no multi-GPU path.", file=sys.stderr)
        return 2

    import torch
    from paper_1604_07893_amd import hyperpower as hpw
    from paper_1604_07893_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    d = inputs.lowrank_svd(M, N, RANK, smin=SMIN, seed=SEED)
    A = torch.from_numpy(d.A).to(dev)
    params = dict(alpha_rule="user", alpha=1.0, variant="stabilised", tol=TOL)
    nbytes = hpw.workspace_bytes(hpw.make_params(**params), M, N)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    X = torch.empty((N, M), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)

    for _ in range(args.warmup):
        hpw.solve(A, out=X, workspace=ws, stream=stream, **params)
    torch.cuda.synchronize()

    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, info = hpw.solve(A, out=X, workspace=ws, stream=stream, time_kernels=True, **params)
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    closed = (d.V / d.s) @ d.U.T
    Xh = X.cpu().numpy()
    err = float(np.linalg.norm(Xh - closed) / np.linalg.norm(closed))

    gflop = sum(i["gflop"] for i in infos)
    gemm_ms = sum(i["gemm_ms"] for i in infos)
    launches = sum(i["gemms"] for i in infos)
    achieved = gflop / gemm_ms if gemm_ms > 0 else 0.0  # GFLOP/ms = TFLOP/s
    last = infos[-1]
    n_stab = last["iters"] - last["switch_iter"] if last["switch_iter"] >= 0 else 0
    n_plain = last["iters"] - n_stab

    line = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "inverses/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "m": M, "n": N, "rank": RANK, "variant": "stabilised",
                   "side": last["side"], "precision": "fp64", "tol": TOL},
        "roofline": {
            "bound": "mfma",
            "kernel": "k_gemm_f64",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": None,
            "gflop_per_launch": gflop / max(launches, 1),
            "avg_launch_ms": gemm_ms / max(launches, 1),
        },
        "gemm_tflops_executed": gflop / (elapsed * 1e3),
        "iters": last["iters"],
        "plain_loops": n_plain,
        "stabilised_loops": n_stab,
        "status": last["status"],
        "rel_err_vs_closed_form": err,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(d, n_plain, n_stab)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
