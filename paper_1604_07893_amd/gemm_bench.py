"""Time the library's MFMA GEMM on given shapes (one JSON line per shape).

    python -m paper_1604_07893_amd.gemm_bench --dtype f64 --shapes 2048x2048x2048,8192x8192x8192

Each product runs `--reps` times after one warm-up, timed with events on the
current stream, through `hp_gemm_ws` with a workspace large enough for every
tile (so split-K tiles run split). `HP_GEMM_TILE` in the environment forces a
tile; otherwise the library's default choice for the shape is used. With
`--check` the result is compared with torch's FP64 product.
"""

from __future__ import annotations

import argparse
import json


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32", "bf16", "f16", "bf16s", "f16s"],
                    help="bf16/f16: FP32 operands rounded while staged; bf16s/f16s: 16-bit "
                         "operands held in memory (A and B^T)")
    ap.add_argument("--shapes", default="2048x2048x2048",
                    help="comma-separated MxNxK list")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--check", action="store_true")
    args = ap.parse_args(argv)

    import torch
    from . import hyperpower as hpw

    dt = torch.float64 if args.dtype == "f64" else torch.float32
    ops = args.dtype if args.dtype in ("bf16", "f16") else None
    torch.manual_seed(args.seed)
    for spec in args.shapes.split(","):
        M, N, K = (int(v) for v in spec.lower().split("x"))
        if args.dtype in ("bf16s", "f16s"):
            h = torch.bfloat16 if args.dtype == "bf16s" else torch.float16
            ldk = -(-K // 8) * 8
            A = torch.randn(M, ldk, device="cuda").to(h)[:, :K]
            Bt = torch.randn(N, ldk, device="cuda").to(h)[:, :K]
            C = torch.empty(M, N, dtype=torch.float32, device="cuda")
            hpw.gemm_bt(A, Bt, out=C)
            torch.cuda.synchronize()
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            for _ in range(args.reps):
                hpw.gemm_bt(A, Bt, out=C)
            e.record()
            torch.cuda.synchronize()
            ms = s.elapsed_time(e) / args.reps
            rec = {"dtype": args.dtype, "M": M, "N": N, "K": K, "ms": ms,
                   "tflops": 2.0 * M * N * K / ms * 1e-9}
            if args.check:
                ref = A.double() @ Bt.double().t()
                rec["max_rel_err"] = float((C.double() - ref).abs().max() / ref.abs().max())
            print(json.dumps(rec), flush=True)
            continue
        vec = 2 if dt == torch.float64 else 4
        lda, ldb = -(-K // vec) * vec, -(-N // vec) * vec
        A = torch.randn(M, lda, dtype=dt, device="cuda")[:, :K]
        B = torch.randn(K, ldb, dtype=dt, device="cuda")[:, :N]
        C = torch.empty(M, N, dtype=dt, device="cuda")
        tiles = -(-M // 128) * -(-N // 128)
        ws = torch.empty(4 * tiles * 128 * 128 * 8 + 4 * 4 * tiles + 4096, dtype=torch.uint8,
                         device="cuda")
        hpw.gemm(A, B, out=C, operands=ops, workspace=ws)
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(args.reps):
            hpw.gemm(A, B, out=C, operands=ops, workspace=ws)
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e) / args.reps
        rec = {"dtype": args.dtype, "M": M, "N": N, "K": K, "ms": ms,
               "tflops": 2.0 * M * N * K / ms * 1e-9}
        if args.check:
            ref = A.double() @ B.double()
            rec["max_rel_err"] = float((C.double() - ref).abs().max() / ref.abs().max())
        print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
