"""The FP64 MFMA GEMM kernel against numpy's FP64 product, elementwise within
the standard error bound |C - C_hat| <= c K u (|A| |B|)."""

import numpy as np
import pytest
import torch

from gpu_common import need_gpu, say, to_dev

pytestmark = pytest.mark.gpu

U64 = 2.0**-53


def even_ld(a):
    """Device copy whose leading dimension is rounded up to an even count (the
    kernel reads 16-byte pairs along rows)."""
    r, c = a.shape
    buf = torch.zeros((r, c + (c & 1)), dtype=torch.float64, device="cuda:0")
    buf[:, :c] = to_dev(a)
    return buf[:, :c]

SHAPES = [
    (1, 1, 1), (16, 16, 4), (128, 128, 16), (127, 129, 17), (200, 200, 100),
    (257, 129, 33), (130, 7, 300), (5, 300, 2), (333, 444, 555), (1024, 1024, 1024),
    (64, 2048, 96),
]


@pytest.mark.parametrize("M,N,K", SHAPES)
def test_gemm_f64_matches_numpy(M, N, K):
    hpw = need_gpu()
    say(f"gemm f64 M={M} N={N} K={K}")
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    C = hpw.gemm(even_ld(A), even_ld(B))
    torch.cuda.synchronize()
    ref = A @ B
    bound = (np.abs(A) @ np.abs(B)) * (2 * K + 4) * U64
    err = np.abs(C.cpu().numpy() - ref)
    assert np.all(err <= bound + 1e-300), float((err / (bound + 1e-300)).max())


def test_gemm_epilogue_identity_and_scale_with_padded_ld():
    hpw = need_gpu()
    rng = np.random.default_rng(5)
    M, K, N = 150, 70, 150
    big = rng.standard_normal((M, K + 10))
    A = to_dev(big)[:, :K]                      # lda = K + 10 (even)
    B = to_dev(rng.standard_normal((K, N)))
    out = torch.full((M, N + 6), 7.0, dtype=torch.float64, device="cuda:0")
    C = hpw.gemm(A, B, alpha=-1.0, beta_identity=1.0, out=out[:, :N])
    torch.cuda.synchronize()
    ref = np.eye(M, N) - big[:, :K] @ B.cpu().numpy()
    assert np.max(np.abs(C.cpu().numpy() - ref)) < 1e-12
    # the padding columns of the output were not touched
    assert torch.all(out[:, N:] == 7.0)


def test_gemm_is_deterministic():
    hpw = need_gpu()
    rng = np.random.default_rng(9)
    A = to_dev(rng.standard_normal((300, 260)))
    B = to_dev(rng.standard_normal((260, 280)))
    c1 = hpw.gemm(A, B).cpu()
    c2 = hpw.gemm(A, B).cpu()
    assert torch.equal(c1, c2)


def test_gemm_rejects_bad_arguments():
    hpw = need_gpu()
    A = torch.zeros((8, 9), dtype=torch.float64, device="cuda:0")   # odd lda
    B = torch.zeros((9, 8), dtype=torch.float64, device="cuda:0")
    with pytest.raises(hpw.HyperpowerError):
        hpw.gemm(A, B)


@pytest.mark.parametrize("M,N,K", [(16, 16, 4), (127, 129, 17), (333, 444, 555), (64, 2048, 96)])
def test_gemm_f32_matches_numpy(M, N, K):
    hpw = need_gpu()
    say(f"gemm f32 M={M} N={N} K={K}")
    rng = np.random.default_rng(M + 5 * N + 11 * K)
    A = rng.standard_normal((M, K)).astype(np.float32)
    B = rng.standard_normal((K, N)).astype(np.float32)
    pad = lambda c: (c + 3) // 4 * 4
    Ad = torch.zeros((M, pad(K)), dtype=torch.float32, device="cuda:0")
    Bd = torch.zeros((K, pad(N)), dtype=torch.float32, device="cuda:0")
    Ad[:, :K] = torch.from_numpy(A).cuda()
    Bd[:, :N] = torch.from_numpy(B).cuda()
    C = hpw.gemm(Ad[:, :K], Bd[:, :N])
    torch.cuda.synchronize()
    ref = A.astype(np.float64) @ B.astype(np.float64)
    bound = (np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64)) * (2 * K + 4) * 2.0**-24
    err = np.abs(C.cpu().numpy().astype(np.float64) - ref)
    assert np.all(err <= bound + 1e-30), float((err / (bound + 1e-30)).max())


@pytest.mark.parametrize("operands", ["bf16", "f16"])
@pytest.mark.parametrize("M,N,K", [(16, 16, 32), (127, 129, 17), (333, 444, 555), (256, 256, 1024)])
def test_gemm_16bit_operands_match_rounded_product(operands, M, N, K):
    """FP32 storage, operands rounded to bf16/fp16 (nearest even), FP32
    accumulation: compare with the FP64 product of the rounded operands."""
    hpw = need_gpu()
    say(f"gemm {operands} M={M} N={N} K={K}")
    rng = np.random.default_rng(M + 3 * N + 7 * K)
    A = rng.standard_normal((M, K)).astype(np.float32)
    B = rng.standard_normal((K, N)).astype(np.float32)
    pad = lambda c: (c + 3) // 4 * 4
    Ad = torch.zeros((M, pad(K)), dtype=torch.float32, device="cuda:0")
    Bd = torch.zeros((K, pad(N)), dtype=torch.float32, device="cuda:0")
    Ad[:, :K] = torch.from_numpy(A).cuda()
    Bd[:, :N] = torch.from_numpy(B).cuda()
    C = hpw.gemm(Ad[:, :K], Bd[:, :N], operands=operands)
    torch.cuda.synchronize()
    tdt = torch.bfloat16 if operands == "bf16" else torch.float16
    Ar = torch.from_numpy(A).to(tdt).double().numpy()
    Br = torch.from_numpy(B).to(tdt).double().numpy()
    ref = Ar @ Br
    bound = (np.abs(Ar) @ np.abs(Br)) * (2 * K + 4) * 2.0**-24
    err = np.abs(C.cpu().numpy().astype(np.float64) - ref)
    assert np.all(err <= bound + 1e-30), float((err / (bound + 1e-30)).max())


def test_autotune_picks_a_tile_and_keeps_results_correct():
    hpw = need_gpu()
    res = hpw.autotune([(512, 512, 512), (300, 200, 100)], dtype="f64", reps=2)
    assert len(res) == 2 and all(r[4] > 0 for r in res)
    table = hpw.tuning_table()
    assert {(r[1], r[2], r[3]) for r in table} >= {(512, 512, 512), (300, 200, 100)}
    rng = np.random.default_rng(3)
    A = rng.standard_normal((300, 100))
    B = rng.standard_normal((100, 200))
    C = hpw.gemm(even_ld(A), even_ld(B))
    ref = A @ B
    bound = (np.abs(A) @ np.abs(B)) * 204 * U64
    assert np.all(np.abs(C.cpu().numpy() - ref) <= bound)


# Products with fewer 128 x 128 output tiles than compute units and a long K
# split K over 4 blocks per tile when a workspace is given (FP64: K >= 1024;
# FP32: K >= 2048 below 128 tiles); ragged shapes leave a short last K-range.
SPLIT_SHAPES = {
    "f64": [(1024, 1024, 2048), (1500, 1400, 1500), (1100, 1300, 2100), (600, 700, 1030)],
    "f32": [(1024, 1024, 2048), (1100, 1300, 2100), (700, 600, 4100)],
}


def _dev_pad(a, dtype):
    vec = 2 if dtype == torch.float64 else 4
    r, c = a.shape
    buf = torch.zeros((r, (c + vec - 1) // vec * vec), dtype=dtype, device="cuda:0")
    buf[:, :c] = torch.from_numpy(a).to(dtype).cuda()
    return buf[:, :c]


@pytest.mark.parametrize("dt,M,N,K", [(d, *s) for d in SPLIT_SHAPES for s in SPLIT_SHAPES[d]])
def test_split_k_gemm_matches_numpy_and_is_reproducible(dt, M, N, K):
    hpw = need_gpu()
    say(f"split-K gemm {dt} M={M} N={N} K={K}")
    assert hpw.gemm_workspace_bytes(M, N, K, dt) > 0
    tdt = torch.float64 if dt == "f64" else torch.float32
    u = U64 if dt == "f64" else 2.0**-24
    rng = np.random.default_rng(M + 13 * N + 17 * K)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    if dt == "f32":
        A, B = A.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64)
    Ad, Bd = _dev_pad(A, tdt), _dev_pad(B, tdt)
    C1 = hpw.gemm(Ad, Bd, workspace=True)
    C2 = hpw.gemm(Ad, Bd, workspace=True)
    C3 = hpw.gemm(Ad, Bd, workspace=True)
    torch.cuda.synchronize()
    # which block of a tile finishes last varies between launches; the sum
    # order does not
    assert torch.equal(C1, C2) and torch.equal(C1, C3)
    ref = A @ B
    bound = (np.abs(A) @ np.abs(B)) * (2 * K + 8) * u
    err = np.abs(C1.cpu().double().numpy() - ref)
    assert np.all(err <= bound + 1e-300), float((err / (bound + 1e-300)).max())


def test_split_k_epilogue_and_undersized_workspace():
    hpw = need_gpu()
    M, N, K = 1536, 1536, 2048          # 144 tiles: splits four ways
    rng = np.random.default_rng(21)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    Ad, Bd = _dev_pad(A, torch.float64), _dev_pad(B, torch.float64)
    C = hpw.gemm(Ad, Bd, alpha=-1.0, beta_identity=1.0, workspace=True)
    ref = np.eye(M, N) - A @ B
    bound = (np.abs(A) @ np.abs(B)) * (2 * K + 8) * U64 + 2 * U64
    assert np.all(np.abs(C.cpu().numpy() - ref) <= bound)
    # too small a workspace: runs unsplit, exactly as hp_gemm does
    small = torch.empty(1024, dtype=torch.uint8, device="cuda:0")
    C_small = hpw.gemm(Ad, Bd, alpha=-1.0, beta_identity=1.0, workspace=small)
    C_plain = hpw.gemm(Ad, Bd, alpha=-1.0, beta_identity=1.0)
    torch.cuda.synchronize()
    assert torch.equal(C_small, C_plain)
    assert hpw.gemm_workspace_bytes(8192, 8192, 8192) == 0    # enough tiles: never splits


def test_two_way_split_from_tuning_table(tmp_path):
    """The two-way split tile, chosen through the handle's tuning table, on a
    ragged FP64 product."""
    import json
    hpw = need_gpu()
    M, N, K = 1280, 1152, 1800
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"rows": [[0, M, N, K, 11]]}))
    hpw.load_tuning(str(path))
    rng = np.random.default_rng(33)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    Ad, Bd = _dev_pad(A, torch.float64), _dev_pad(B, torch.float64)
    ws = torch.empty(2 * 10 * 9 * 128 * 128 * 8 + 4096, dtype=torch.uint8, device="cuda:0")
    C1 = hpw.gemm(Ad, Bd, workspace=ws)
    C2 = hpw.gemm(Ad, Bd, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
    ref = A @ B
    bound = (np.abs(A) @ np.abs(B)) * (2 * K + 8) * U64
    assert np.all(np.abs(C1.cpu().numpy() - ref) <= bound)


def _h16(a, dt, pad=8):
    r, c = a.shape
    buf = torch.zeros((r, (c + pad - 1) // pad * pad), dtype=dt, device="cuda:0")
    buf[:, :c] = torch.from_numpy(a).to(dt).cuda()
    return buf[:, :c]


@pytest.mark.parametrize("dt", [torch.bfloat16, torch.float16])
@pytest.mark.parametrize("M,N,K,tile", [(16, 16, 32, None), (127, 129, 17, None), (333, 444, 555, None),
                                        (1024, 1024, 1024, None), (600, 520, 200, 14),
                                        (530, 610, 300, 15), (700, 300, 100, 4), (300, 700, 90, 2),
                                        (600, 520, 256, 16), (530, 610, 320, 17),
                                        (300, 280, 200, 17)])
def test_gemm_16bit_operands_in_memory(dt, M, N, K, tile, tmp_path):
    """HP_DTYPE_BF16 / HP_DTYPE_F16: A and B^T held in 16 bits, FP32
    accumulation: compare with the FP64 product of the same 16-bit values
    (every tile configuration of the kernel, ragged shapes)."""
    import json
    hpw = need_gpu()
    say(f"gemm h16 {dt} M={M} N={N} K={K} tile={tile}")
    if tile is not None:
        code = 4 if dt == torch.bfloat16 else 5
        path = tmp_path / "tune.json"
        path.write_text(json.dumps({"rows": [[code, M, N, K, tile]]}))
        hpw.load_tuning(str(path))
    rng = np.random.default_rng(M + 3 * N + 5 * K)
    A = rng.standard_normal((M, K))
    Bt = rng.standard_normal((N, K))
    Ad, Btd = _h16(A, dt), _h16(Bt, dt)
    C = hpw.gemm_bt(Ad, Btd)
    C2 = hpw.gemm_bt(Ad, Btd)
    torch.cuda.synchronize()
    assert torch.equal(C, C2)
    Ar = Ad.double().cpu().numpy()
    Br = Btd.double().cpu().numpy().T
    ref = Ar @ Br
    bound = (np.abs(Ar) @ np.abs(Br)) * (2 * K + 4) * 2.0**-24
    err = np.abs(C.cpu().numpy().astype(np.float64) - ref)
    assert np.all(err <= bound + 1e-30), float((err / (bound + 1e-30)).max())



# The 4-wave FP64 tile filled by load-to-LDS (tile 19), forced through the
# tuning table: ragged M and N, a single K-tile, N = 2, and two shapes it hands
# to the 16-wave kernel on the same tiles (K not a multiple of 16, odd N).
DMA_TILE = 19


@pytest.mark.parametrize("M,N,K", [(256, 256, 16), (300, 260, 48), (130, 2, 32), (1000, 1002, 1024),
                                   (512, 384, 100), (300, 259, 64)])
def test_gemm_f64_load_to_lds_tile(M, N, K, tmp_path):
    import json
    hpw = need_gpu()
    say(f"gemm f64 load-to-LDS tile M={M} N={N} K={K}")
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"rows": [[0, M, N, K, DMA_TILE]]}))
    hpw.load_tuning(str(path))
    rng = np.random.default_rng(M + 13 * N + 17 * K)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    Ad, Bd = _dev_pad(A, torch.float64), _dev_pad(B, torch.float64)
    C1 = hpw.gemm(Ad, Bd)
    C2 = hpw.gemm(Ad, Bd, alpha=-1.0, beta_identity=1.0)
    torch.cuda.synchronize()
    ref = A @ B
    bound = (np.abs(A) @ np.abs(B)) * (2 * K + 4) * U64
    err = np.abs(C1.cpu().numpy() - ref)
    assert np.all(err <= bound + 1e-300), float((err / (bound + 1e-300)).max())
    # the epilogue's identity and scale on the same tile: exactly I - C1
    assert torch.equal(C2, torch.eye(M, N, dtype=torch.float64, device="cuda:0") - C1)


def test_solve_on_the_load_to_lds_tile_matches_the_16_wave_tile(tmp_path):
    """A 3072^2 FP64 solve (576 tiles per product: the load-to-LDS tile by
    default) against the same solve with the 16-wave tile forced: same loop
    count, X equal to rounding, and A X = I to 1e-10."""
    import json
    hpw = need_gpu()
    n = 3072
    say(f"solve f64 {n}^2 load-to-LDS tile vs 16-wave tile")
    g = torch.Generator(device="cuda:0").manual_seed(3072)
    A = torch.randn((n, n), dtype=torch.float64, device="cuda:0", generator=g) / n**0.5
    A += 2.0 * torch.eye(n, dtype=torch.float64, device="cuda:0")   # singular values in ~[1, 3]
    X1, info1 = hpw.solve(A, tol=1e-12)
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"rows": [[0, n, n, n, 13]]}))
    hpw.load_tuning(str(path))
    try:
        X2, info2 = hpw.solve(A, tol=1e-12)
    finally:
        path.write_text(json.dumps({"rows": [[0, n, n, n, DMA_TILE]]}))
        hpw.load_tuning(str(path))
    torch.cuda.synchronize()
    assert info1["status"] == info2["status"] == "ok"
    assert info1["iters"] == info2["iters"]
    scale = float(X2.abs().max())
    assert float((X1 - X2).abs().max()) <= 1e-12 * scale
    I = torch.eye(n, dtype=torch.float64, device="cuda:0")
    assert float((A @ X1 - I).abs().max()) <= 1e-10


# The 4-wave FP32 tile of 128 x 128 per wave (tile 20, 256 x 256 tiles,
# load-to-LDS), forced through the tuning table: a single K-tile, ragged M and
# N, and shapes it hands to a register-staged kernel on the same tiles (N not a
# multiple of 4, K not a multiple of 32).
F32_DMA_TILE = 20


@pytest.mark.parametrize("M,N,K", [(256, 256, 32), (300, 260, 64), (520, 1000, 96), (1000, 1004, 1024),
                                   (300, 258, 64), (512, 384, 100)])
def test_gemm_f32_load_to_lds_tile(M, N, K, tmp_path):
    import json
    hpw = need_gpu()
    say(f"gemm f32 load-to-LDS tile M={M} N={N} K={K}")
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"rows": [[1, M, N, K, F32_DMA_TILE]]}))
    hpw.load_tuning(str(path))
    rng = np.random.default_rng(M + 19 * N + 23 * K)
    A = rng.standard_normal((M, K)).astype(np.float32)
    B = rng.standard_normal((K, N)).astype(np.float32)
    Ad, Bd = _dev_pad(A.astype(np.float64), torch.float32), _dev_pad(B.astype(np.float64), torch.float32)
    C1 = hpw.gemm(Ad, Bd)
    C2 = hpw.gemm(Ad, Bd, alpha=-1.0, beta_identity=1.0)
    torch.cuda.synchronize()
    ref = A.astype(np.float64) @ B.astype(np.float64)
    bound = (np.abs(A).astype(np.float64) @ np.abs(B).astype(np.float64)) * (2 * K + 4) * 2.0**-24
    err = np.abs(C1.cpu().numpy().astype(np.float64) - ref)
    assert np.all(err <= bound + 1e-30), float((err / (bound + 1e-30)).max())
    assert torch.equal(C2, torch.eye(M, N, dtype=torch.float32, device="cuda:0") - C1)
