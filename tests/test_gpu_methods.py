"""The comparison schemes of Sections 1.3 and 2 (SM, CM, FM, HM) and PM on the
GPU (hp_params.method) against the same schemes in the CPU oracle.

Bar as for PM: relative Frobenius difference from the oracle's X <= 1e-10 in
FP64, the same loop count, the same relative changes above the rounding floor,
and the executed product count of each scheme per loop.
"""

import numpy as np
import pytest
import torch

import oracle as O
from gpu_common import need_gpu, rel, say, to_dev
from paper_1604_07893_amd import inputs

pytestmark = pytest.mark.gpu

METHODS = ["sm", "cm", "fm", "hm", "pm"]
PRODUCTS = {"sm": 2, "cm": 3, "fm": 5, "hm": 9, "pm": 7}


def run(A, **kw):
    hpw = need_gpu()
    X, info = hpw.solve(to_dev(A), **kw)
    torch.cuda.synchronize()
    return X.cpu().numpy(), info


@pytest.mark.parametrize("side", ["right", "left"])
@pytest.mark.parametrize("method", METHODS)
def test_method_matches_oracle_uniform(method, side):
    say(f"method {method} side {side}")
    A = inputs.uniform(200, 100, seed=1001)
    ref = O.solve(A, kind="mp", method=method, tol=1e-12)
    X, info = run(A, method=method, tol=1e-12, side=side)
    assert info["status"] == ref.status == "ok"
    assert info["iters"] == ref.iters
    assert info["gemms"] == PRODUCTS[method] * info["iters"]
    assert rel(X, ref.X) <= 1e-10
    d_got = np.array(info["d_hist"])
    d_ref = np.array(ref.d_hist[:len(d_got)])
    big = d_ref > 1e-13
    np.testing.assert_allclose(d_got[big], d_ref[big], rtol=1e-6)
    for r in O.penrose_residuals(A, X):
        assert r < 1e-12


@pytest.mark.parametrize("method", METHODS)
def test_method_paper_rule_on_square_input(method):
    """Rule (stopreliable) divides by p^k alpha with the scheme's own order p."""
    say(f"method {method} paper_4_1")
    d = inputs.square_svd(160, smin=1e-2, seed=77)
    ref = O.solve(d.A, kind="mp", method=method, stop="paper_4_1", tol=1e-8)
    X, info = run(d.A, method=method, stop="paper_4_1", tol=1e-8)
    assert info["status"] == ref.status
    assert info["iters"] == ref.iters
    assert rel(X, ref.X) <= 1e-10


@pytest.mark.parametrize("method", ["sm", "fm", "hm"])
def test_method_drazin_and_stabilised(method):
    say(f"method {method} drazin + stabilised")
    # tol 3e-10 sits at least 2x away from every relative change of these runs
    # (near 1e-11 the nilpotent part's rounding moves the change by tens of %)
    dz = inputs.drazin_jordan(n=96, nb=80, seed=5)
    ref = O.solve(dz.A, kind="drazin", l=dz.index, method=method, variant="stabilised", tol=3e-10)
    X, info = run(dz.A, kind="drazin", l=dz.index, method=method, variant="stabilised", tol=3e-10)
    assert info["status"] == ref.status
    assert info["iters"] == ref.iters and info["switch_iter"] == ref.switch_iter
    assert rel(X, ref.X) <= 1e-10
    lr = inputs.lowrank_svd(240, 120, 80, smin=1e-3, seed=6)
    ref = O.solve(lr.A, kind="mp", method=method, variant="stabilised", tol=1e-10)
    X, info = run(lr.A, method=method, variant="stabilised", tol=1e-10)
    assert info["status"] == ref.status == "ok"
    assert info["iters"] == ref.iters
    assert rel(X, ref.X) <= 1e-9


def test_method_fp32_and_unsupported_combinations():
    hpw = need_gpu()
    A = inputs.uniform(150, 90, seed=12)
    ref = O.solve(A, kind="mp", method="cm", tol=1e-12)
    X, info = run(A, method="cm", precision="fp32", tol=1e-5)
    assert info["status"] in ("ok", "stagnated")
    assert rel(X, ref.X) <= 1e-4
    with pytest.raises(hpw.HyperpowerError):
        run(A, method="sm", precision="mixed")
    with pytest.raises(hpw.HyperpowerError):
        hpw.solve_batched([to_dev(A)], method="hm")


@pytest.mark.parametrize("method", ["sm", "cm", "hm", "pm"])
def test_hilbert_example_8_2_matches_oracle(method):
    """Example 8.2's setting on H_{100x90}: X0 = 2/(sigma_1^2 + sigma_r^2) H^T
    (the oracle's SVD gives alpha; the GPU is handed the same value), rule
    (stopreliable) with eps = 1e-5. kappa(H) is near 1e17, so iterates past
    the first loops carry rounding amplified by it: the loop count and the
    first relative changes are compared exactly / to 1e-6, X to 1e-5 (a
    1e-14 change of alpha alone moves the oracle's own X by ~4e-8)."""
    say(f"hilbert 100x90 {method}")
    H = inputs.hilbert(100, 90)
    ref = O.solve(H, kind="mp", method=method, alpha_rule="sigma_opt", stop="paper_4_1", tol=1e-5)
    X, info = run(H, method=method, alpha_rule="user", alpha=float(ref.alpha), stop="paper_4_1",
                  tol=1e-5)
    assert info["status"] == ref.status == "ok"
    assert info["iters"] == ref.iters
    np.testing.assert_allclose(info["d_hist"][:5], ref.d_hist[:5], rtol=1e-6)
    assert rel(X, ref.X) <= 1e-5
