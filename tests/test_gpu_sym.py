"""Symmetric products (hp_gemm_sym) and the solves that use them.

When X_k = p(A^T A) A^T (Moore-Penrose from X0 = alpha A^T), R = I - X A (or
I - A X) is symmetric, and so is every product of a loop formed from R alone
(Section 2's factored polynomial) and the middle product X A of the
stabilised step (Section 7). With HP_FLAG_SYMMETRIC (inputs whose rank equals
the residual's side) those launches compute the upper triangle's tiles only
and mirror them. Checked here: the kernel against a plain FP64
product on the host (ragged sizes, split tiles, both element types, alpha and
the identity term, no workspace, calls in a row), and solves with and without
the symmetric launches (same loop counts, both at the closed-form inverse to
1e-10)."""

import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from gpu_common import need_gpu, rel, say, to_dev
from paper_1604_07893_amd import inputs

pytestmark = pytest.mark.gpu


def gram(N, K, seed, dtype):
    g = np.random.default_rng(seed).standard_normal((N, K))
    G = torch.from_numpy(g).to(dtype).cuda()
    return g, G, G.t().contiguous()


@pytest.mark.parametrize("N,K,dtype", [
    (300, 200, torch.float64),     # 3 x 3 tiles, ragged N and K: 6 tiles, pieces split
    (2100, 1000, torch.float64),   # 17 x 17 tiles (153), ragged tail
    (2048, 4096, torch.float64),   # the residual's shape in the 4096 x 2048 workload
    (776, 332, torch.float32),     # rows of 16 bytes: N, K multiples of 4
    (3000, 700, torch.float32),
])
def test_sym_product_matches_host_product(N, K, dtype):
    hpw = need_gpu()
    say(f"gemm_sym N={N} K={K} {dtype}")
    g, G, Gt = gram(N, K, 5000 + N, dtype)
    C = hpw.gemm_sym(G, Gt, alpha=0.5, beta_identity=2.0)
    torch.cuda.synchronize()
    c = C.cpu().numpy()
    # exactly symmetric: each (i, j), i <= j, formed once and stored twice
    assert np.array_equal(c, c.T)
    gd = G.double().cpu().numpy()  # the operands as the kernel saw them
    ref = 0.5 * (gd @ gd.T) + 2.0 * np.eye(N)
    tol = 1e-14 if dtype == torch.float64 else 2e-6
    assert np.abs(c - ref).max() <= tol * np.sqrt(K) * np.abs(ref).max()
    # the full product of the same kernel family agrees to rounding
    F = hpw.gemm(G, Gt, alpha=0.5, beta_identity=2.0)
    torch.cuda.synchronize()
    f = F.cpu().numpy()
    assert np.abs(np.triu(c) - np.triu(f)).max() <= tol * np.sqrt(K) * np.abs(ref).max()


def test_sym_product_without_workspace_is_full_product():
    hpw = need_gpu()
    say("gemm_sym without workspace")
    g, G, Gt = gram(500, 300, 77, torch.float64)
    C = hpw.gemm_sym(G, Gt, workspace=False)
    torch.cuda.synchronize()
    assert np.abs(C.cpu().numpy() - g @ g.T).max() <= 1e-12 * np.abs(g @ g.T).max()


def test_sym_calls_in_a_row_share_a_workspace():
    """The arrival counters are cleared by every call and left zero by every
    launch: a second, smaller product in the same workspace is right."""
    hpw = need_gpu()
    say("gemm_sym twice, one workspace")
    lib = hpw.load_library()
    sz = ctypes.c_size_t()
    assert lib.hp_gemm_sym_workspace_bytes(0, 2100, 1000, ctypes.byref(sz)) == 0
    ws = torch.empty(max(sz.value, 256), dtype=torch.uint8, device="cuda")
    for N, K, seed in ((2100, 1000, 1), (640, 900, 2), (2100, 1000, 3)):
        g, G, Gt = gram(N, K, seed, torch.float64)
        C = hpw.gemm_sym(G, Gt, workspace=ws)
        torch.cuda.synchronize()
        ref = g @ g.T
        assert np.abs(C.cpu().numpy() - ref).max() <= 1e-14 * np.sqrt(K) * np.abs(ref).max()


def test_sym_rejects_other_dtypes_and_shapes():
    hpw = need_gpu()
    G = torch.zeros((64, 32), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        hpw.gemm_sym(G, G)  # B must be K x N
    lib = hpw.load_library()
    sz = ctypes.c_size_t()
    assert lib.hp_gemm_sym_workspace_bytes(4, 64, 32, ctypes.byref(sz)) == hpw.HP_EINVAL


@pytest.mark.parametrize("m,n,variant,stop", [
    (2100, 2100, "plain", "rel_fro"),         # square, s = 2100: 17 x 17 tiles, ragged
    (2300, 2100, "stabilised", "rel_fro"),    # left form, s = 2100; the middle product X A too
    (2100, 2300, "stabilised", "rel_fro"),    # right form, s = 2100; the middle product A X
    (2100, 2100, "plain", "rel_fro_bound"),   # the residual check forms the full R
])
def test_solve_symmetric_matches_full_products(m, n, variant, stop):
    """With HP_FLAG_SYMMETRIC the loop's s x s products run symmetric
    (full-rank inputs); by default every product is formed in full. Same loop counts,
    both at the closed-form inverse to 1e-10, the symmetric one no less
    accurate."""
    hpw = need_gpu()
    say(f"solve sym vs full {m}x{n} {variant} {stop}")
    d = inputs.lowrank_svd(m, n, min(m, n), smin=1e-3, seed=4242)
    closed = (d.V / d.s) @ d.U.T
    A = to_dev(d.A)
    kw = dict(alpha_rule="user", alpha=1.0, variant=variant, tol=1e-10, stop=stop)
    Xs, i_s = hpw.solve(A, symmetric=True, **kw)
    Xf, i_f = hpw.solve(A, **kw)
    torch.cuda.synchronize()
    assert i_s["status"] == i_f["status"] == "ok"
    assert i_s["gemms_sym"] > 0 and i_f["gemms_sym"] == 0
    assert i_s["switch_iter"] == i_f["switch_iter"]
    if stop == "rel_fro":
        assert i_s["iters"] == i_f["iters"]
    else:
        # the residual check reads the full R, which still holds the part the
        # symmetric loops left (rounding level): it may ask for one more,
        # low-order loop before it settles
        assert i_f["iters"] <= i_s["iters"] <= i_f["iters"] + 1
    xs, xf = Xs.cpu().numpy(), Xf.cpu().numpy()
    es, ef, dsf = rel(xs, closed), rel(xf, closed), rel(xs, xf)
    say(f"  iters {i_s['iters']}: err sym {es:.2e}, full {ef:.2e}, sym vs full {dsf:.2e}")
    # both at the inverse to the method's tolerance; the two differ by the
    # rounding of the summation order, amplified as any rounding is (kappa 1e3)
    assert es <= 1e-10 and ef <= 1e-10 and dsf <= 1e-10
    assert es <= 2.0 * ef + 1e-11
    # the symmetric launches count N (N + 1) K flops each
    assert i_s["gflop"] < i_f["gflop"]
    if m == n and stop == "rel_fro":
        # and the FP64 oracle (right form, full products) takes the same loops
        ref = O.solve(d.A, kind="mp", alpha_rule="user", alpha=1.0, variant=variant, tol=1e-10)
        say(f"  oracle iters {ref.iters}, sym vs oracle {rel(xs, ref.X):.2e}")
        assert ref.iters == i_s["iters"]
        assert rel(xs, ref.X) <= 1e-10


def test_solve_with_user_x0_or_drazin_keeps_full_products():
    """A caller's X0 (not alpha A^T) and the Drazin kind give no symmetric R:
    no symmetric launches even with HP_FLAG_SYMMETRIC."""
    hpw = need_gpu()
    say("no sym for user X0 / drazin")
    d = inputs.square_svd(2100, smin=1e-2, seed=99)
    A = to_dev(d.A)
    X0 = (A.t() / float(d.s.max() ** 2)).contiguous()
    _, info = hpw.solve(A, X0=X0, tol=1e-8, symmetric=True)
    assert info["gemms_sym"] == 0
    dz = inputs.drazin_jordan(n=2048, nb=1792, cond_p=10.0, seed=1004)
    _, info = hpw.drazin(to_dev(dz.A), 3, tol=1e-8, symmetric=True)
    assert info["gemms_sym"] == 0


@pytest.mark.parametrize("precision", ["mixed", "fp32_fp64"])
def test_staged_solves_with_symmetric_products(precision):
    """HP_FLAG_SYMMETRIC in staged solves. Mirroring the upper triangle turns
    the part of R that is not symmetric into a symmetric error of the same
    size, which grows by the order per loop in the unconverged directions:
    harmless from FP64 rounding over a few loops, not from FP32 or 16-bit
    rounding (rules that let FP32 loops run symmetric diverged, to 1e50 and
    1e67 on this input). Staged solves therefore form full products: no
    symmetric launches, the same result as without the flag."""
    hpw = need_gpu()
    say(f"{precision} sym 2100")
    d = inputs.square_svd(2100, smin=1e-3, seed=31)
    closed = (d.V / d.s) @ d.U.T
    A = to_dev(d.A)
    kw = dict(alpha_rule="user", alpha=1.0, precision=precision, tol=1e-10)
    Xs, i_s = hpw.solve(A, symmetric=True, **kw)
    Xf, i_f = hpw.solve(A, **kw)
    torch.cuda.synchronize()
    es, ef = rel(Xs.cpu().numpy(), closed), rel(Xf.cpu().numpy(), closed)
    say(f"  stages {i_s['iters_stage']} vs {i_f['iters_stage']}, sym launches {i_s['gemms_sym']}, "
        f"err {es:.2e} vs {ef:.2e}")
    assert i_s["status"] == i_f["status"] == "ok"
    assert i_f["gemms_sym"] == 0
    assert i_s["gemms_sym"] == 0
    assert es <= 1e-10 and es <= 2.0 * ef + 1e-11


def test_complex_solve_with_symmetric_products():
    """A complex full-rank 1100 x 1100 A: the real form (2200 x 2200) with
    X0 = alpha times its transpose keeps X A symmetric, so HP_FLAG_SYMMETRIC
    applies to hp_solve_complex too; same loops and the same inverse
    (LAPACK's complex pseudo-inverse) as without it."""
    hpw = need_gpu()
    say("complex 1100 sym")
    rng = np.random.default_rng(1100)
    A = (rng.standard_normal((1100, 1100)) + 1j * rng.standard_normal((1100, 1100))) / 40.0
    alpha = 1.0 / np.linalg.svd(A, compute_uv=False)[0] ** 2
    Ad = torch.from_numpy(A).cuda()
    kw = dict(alpha_rule="user", alpha=alpha, tol=1e-10)
    Xs, i_s = hpw.solve_complex(Ad, symmetric=True, **kw)
    Xf, i_f = hpw.solve_complex(Ad, **kw)
    torch.cuda.synchronize()
    P = np.linalg.pinv(A)
    es, ef = rel(Xs.cpu().numpy(), P), rel(Xf.cpu().numpy(), P)
    say(f"  iters {i_s['iters']} / {i_f['iters']}, sym launches {i_s['gemms_sym']}, "
        f"err {es:.2e} vs {ef:.2e}")
    assert i_s["status"] == i_f["status"] == "ok"
    assert i_s["gemms_sym"] > 0 and i_f["gemms_sym"] == 0
    assert i_s["iters"] == i_f["iters"]
    assert es <= 1e-10 and es <= 2.0 * ef + 1e-11


def test_symmetric_products_with_gpu_alpha():
    """X0 = alpha A^T with alpha from the GPU power iteration (sigma_max2) is
    as symmetric as a given alpha: the same loops and the same inverse with and
    without the symmetric products."""
    hpw = need_gpu()
    say("sym with sigma_max2 alpha")
    d = inputs.lowrank_svd(2100, 2100, 2100, smin=1e-3, seed=77)
    closed = (d.V / d.s) @ d.U.T
    A = to_dev(d.A)
    kw = dict(alpha_rule="sigma_max2", tol=1e-10)
    Xs, i_s = hpw.solve(A, symmetric=True, **kw)
    Xf, i_f = hpw.solve(A, **kw)
    torch.cuda.synchronize()
    es, ef = rel(Xs.cpu().numpy(), closed), rel(Xf.cpu().numpy(), closed)
    say(f"  alpha {i_s['alpha']:.6f}, iters {i_s['iters']} / {i_f['iters']}, "
        f"sym launches {i_s['gemms_sym']}, err {es:.2e} vs {ef:.2e}")
    assert i_s["alpha"] == i_f["alpha"]
    assert i_s["status"] == i_f["status"] == "ok"
    assert i_s["gemms_sym"] > 0 and i_s["iters"] == i_f["iters"]
    assert es <= 1e-10 and es <= 2.0 * ef + 1e-11


@pytest.mark.parametrize("N,K", [
    (7000, 512),    # 55 x 55 tiles (1540 >= 3 rounds of 512 blocks): k_gemm_w4dma_sym,
                    # 2 rounds of whole tiles, the ragged rest split by K-steps
    (300, 208),     # 6 triangle tiles, under 3 rounds: the 16-wave stream-K launch
    (2100, 1024),   # 153 triangle tiles: likewise
    (512, 100),     # K not a multiple of 16: likewise
])
def test_sym_product_on_the_load_to_lds_tile(N, K, tmp_path):
    """Symmetric products with the 4-wave load-to-LDS tile chosen (tile 19,
    forced through the tuning table): its stream-K form where the triangle
    fills three rounds of the device's blocks, the 16-wave stream-K kernel
    otherwise. Exactly symmetric, within the product's bound of the host
    product, to rounding the full product; two calls in a row give the same
    bits."""
    import json
    hpw = need_gpu()
    say(f"gemm_sym load-to-LDS tile N={N} K={K}")
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"rows": [[0, N, N, K, 19]]}))
    hpw.load_tuning(str(path))
    g, G, Gt = gram(N, K, 7000 + N, torch.float64)
    C = hpw.gemm_sym(G, Gt, alpha=0.5, beta_identity=2.0)
    C2 = hpw.gemm_sym(G, Gt, alpha=0.5, beta_identity=2.0)
    F = hpw.gemm(G, Gt, alpha=0.5, beta_identity=2.0)
    torch.cuda.synchronize()
    assert torch.equal(C, C2)
    c, f = C.cpu().numpy(), F.cpu().numpy()
    assert np.array_equal(c, c.T)
    ref = 0.5 * (g @ g.T) + 2.0 * np.eye(N)
    tol = 1e-14 * np.sqrt(K) * np.abs(ref).max()
    assert np.abs(c - ref).max() <= tol
    assert np.abs(np.triu(c) - np.triu(f)).max() <= tol


def test_solve_symmetric_beside_the_load_to_lds_tile():
    """3072^2 (576 tiles per product: full products on the load-to-LDS tile,
    symmetric ones on its stream-K form) with HP_FLAG_SYMMETRIC against the
    same solve with full products: same loops, both at the closed-form
    inverse to 1e-10."""
    hpw = need_gpu()
    say("solve sym vs full 3072^2 load-to-LDS tile")
    d = inputs.lowrank_svd(3072, 3072, 3072, smin=1e-3, seed=3072)
    closed = (d.V / d.s) @ d.U.T
    A = to_dev(d.A)
    kw = dict(alpha_rule="user", alpha=1.0, tol=1e-10)
    Xs, i_s = hpw.solve(A, symmetric=True, **kw)
    Xf, i_f = hpw.solve(A, **kw)
    torch.cuda.synchronize()
    assert i_s["status"] == i_f["status"] == "ok"
    assert i_s["gemms_sym"] > 0 and i_f["gemms_sym"] == 0
    assert i_s["iters"] == i_f["iters"]
    xs, xf = Xs.cpu().numpy(), Xf.cpu().numpy()
    es, ef = rel(xs, closed), rel(xf, closed)
    say(f"  iters {i_s['iters']}: err sym {es:.2e}, full {ef:.2e}")
    assert es <= 1e-10 and ef <= 1e-10 and es <= 2.0 * ef + 1e-11
