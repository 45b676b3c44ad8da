"""Example 8.3 on the GPU: X0 = diag(1/a_ii) (choice3), loops with Chop at the
end of each one (hp_params.alpha_rule = HP_ALPHA_DIAG, hp_params.chop), on the
seeded 841 x 841 grid-stencil stand-in for the paper's sparse matrix; and other
outer inverses A^(2)_{T,S} from a user-supplied X0 = alpha G (weighted
Moore-Penrose, group, Bott-Duffin), all against the CPU oracle.

Chop makes an entry zero or not by comparing it with the threshold. The GPU
and the oracle must agree entrywise to TOL = 1e-12 max|X|; every unchopped
entry of these cases is checked to lie more than 10 TOL from the threshold
(the closest is 6e-12 against TOL ~ 3e-13), so the two cannot chop
differently: the zero patterns must then match exactly.
"""

import numpy as np
import pytest
import torch

import oracle as O
from gpu_common import need_gpu, rel, say, to_dev
from paper_1604_07893_amd import inputs

pytestmark = pytest.mark.gpu

EPS = 1e-5
STEP = {"pm": 18, "sm": 2, "cm": 3}


def run(A, **kw):
    hpw = need_gpu()
    X, info = hpw.solve(to_dev(A), **kw)
    torch.cuda.synchronize()
    return X.cpu().numpy(), info


def test_diag_x0_converges_to_the_inverse():
    say("diag x0 400")
    A = inputs.grid_stencil(side=20)
    ref = O.solve(A, kind="mp", alpha_rule="diag", tol=1e-12)
    X, info = run(A, alpha_rule="diag", tol=1e-12)
    assert info["status"] == ref.status == "ok"
    assert info["iters"] == ref.iters and info["alpha"] == 1.0
    assert rel(X, ref.X) <= 1e-12
    assert rel(X, np.linalg.inv(A)) <= 1e-12


@pytest.mark.parametrize("method,loops", [("pm", 1), ("pm", 2), ("cm", 3), ("sm", 5)])
def test_chopped_preconditioner_matches_oracle(method, loops):
    """X_1 of PM, X_3 of CM, X_5 of SM with Chop[X, 1e-5] after each loop
    (the preconditioners compared in Example 8.3)."""
    say(f"precond {method} x{loops}")
    A = inputs.grid_stencil()
    X = np.diag(1.0 / np.diag(A))
    ref = O.solve(A, kind="mp", alpha_rule="diag", method=method, max_iter=loops, chop_eps=EPS)
    tol = 1e-12 * np.max(np.abs(ref.X))
    for _ in range(loops):          # the margin of every loop's unchopped iterate
        pre = O.hyperpower_direct_step(A, X, STEP[method])
        assert float(np.min(np.abs(np.abs(pre) - EPS))) > 10 * tol
        X = np.where(np.abs(pre) < EPS, 0.0, pre)
    Xg, info = run(A, alpha_rule="diag", method=method, max_iter=loops, chop=EPS)
    assert info["status"] == "maxiter" and info["iters"] == loops
    assert np.array_equal(Xg == 0, ref.X == 0)
    assert 0 < np.count_nonzero(Xg) < Xg.size
    assert np.max(np.abs(Xg - ref.X)) <= tol
    np.testing.assert_allclose(info["d_hist"][:loops], ref.d_hist, rtol=1e-10)


def test_chop_in_fp32_and_rejected_combinations():
    hpw = need_gpu()
    A = inputs.grid_stencil(side=12)
    ref = O.solve(A, kind="mp", alpha_rule="diag", max_iter=1, chop_eps=EPS)
    X, info = run(A, alpha_rule="diag", max_iter=1, chop=EPS, precision="fp32")
    assert info["iters"] == 1
    assert rel(X, ref.X) <= 1e-5
    with pytest.raises(hpw.HyperpowerError):
        run(A, alpha_rule="diag", chop=EPS, precision="mixed")
    with pytest.raises(hpw.HyperpowerError):
        run(A, chop=EPS, stop="rel_fro_bound")
    with pytest.raises(hpw.HyperpowerError):
        run(inputs.uniform(60, 40, seed=3), alpha_rule="diag")
    with pytest.raises(hpw.HyperpowerError):
        hpw.solve_batched([to_dev(A)], chop=EPS)


def test_weighted_moore_penrose_from_user_g():
    say("weighted mp")
    rng = np.random.default_rng(3)
    m, n = 200, 120
    A = rng.standard_normal((m, n))
    Mw, Nw = inputs.spd(m, 5.0, seed=11), inputs.spd(n, 5.0, seed=12)
    G = np.linalg.solve(Nw, A.T @ Mw)
    alpha = 1.0 / np.max(np.linalg.eigvals(G @ A).real)
    ref = O.solve(A, X0=alpha * G, alpha=alpha, tol=1e-12)
    X, info = run(A, X0=to_dev(alpha * G), alpha=alpha, tol=1e-12)
    assert info["status"] == ref.status == "ok" and info["iters"] == ref.iters
    assert rel(X, ref.X) <= 1e-10
    MAX = Mw @ A @ X
    assert np.linalg.norm(MAX - MAX.T) / np.linalg.norm(MAX) < 1e-10


def test_group_inverse_on_gpu():
    say("group inverse")
    dz = inputs.drazin_jordan(n=160, nb=120, block=1, seed=8)
    ref = O.solve(dz.A, kind="drazin", l=1, variant="stabilised", tol=1e-11)
    X, info = run(dz.A, kind="drazin", l=1, variant="stabilised", tol=1e-11)
    assert info["status"] == ref.status == "ok" and info["iters"] == ref.iters
    assert rel(X, ref.X) <= 1e-10
    A = dz.A
    assert np.linalg.norm(A @ X - X @ A) / np.linalg.norm(A @ X) < 1e-10


def test_bott_duffin_inverse_on_gpu():
    say("bott-duffin")
    rng = np.random.default_rng(21)
    n, k = 160, 100
    A = inputs.spd(n, 20.0, seed=13) + 0.05 * rng.standard_normal((n, n))
    QL = inputs.haar_columns(rng, n, k)
    PL = QL @ QL.T
    alpha = 1.0 / np.max(np.abs(np.linalg.eigvals(PL @ A)))
    ref = O.solve(A, X0=alpha * PL, alpha=alpha, variant="stabilised", tol=1e-12)
    X, info = run(A, X0=to_dev(alpha * PL), alpha=alpha, variant="stabilised", tol=1e-12)
    assert info["status"] == ref.status == "ok" and info["iters"] == ref.iters
    assert rel(X, ref.X) <= 1e-10
    closed = PL @ np.linalg.inv(A @ PL + (np.eye(n) - PL))
    assert rel(X, closed) <= 1e-10
