"""Complex A on the GPU (hp_solve_complex: the loop on the real form
[[Re A, -Im A], [Im A, Re A]]) against the oracle run in complex arithmetic
with the same alpha, and against LAPACK's complex pseudo-inverse."""

import numpy as np
import pytest
import torch

import oracle as O
from gpu_common import need_gpu, rel, say

pytestmark = pytest.mark.gpu


def complex_input(m, n, rank, seed):
    rng = np.random.default_rng(seed)
    G1 = rng.standard_normal((m, rank)) + 1j * rng.standard_normal((m, rank))
    G2 = rng.standard_normal((rank, n)) + 1j * rng.standard_normal((rank, n))
    return G1 @ G2 / np.sqrt(rank)


@pytest.mark.parametrize("m,n,rank,variant", [(120, 80, 80, "plain"), (80, 120, 80, "plain"),
                                              (100, 100, 60, "stabilised"),
                                              (257, 130, 90, "stabilised")])
def test_complex_moore_penrose_matches_oracle(m, n, rank, variant):
    hpw = need_gpu()
    say(f"complex {m}x{n} rank {rank} {variant}")
    A = complex_input(m, n, rank, seed=m + 7 * n + rank)
    alpha = 1.0 / np.linalg.svd(A, compute_uv=False)[0] ** 2
    ref = O.solve(A, kind="mp", alpha_rule="user", alpha=alpha, variant=variant, tol=1e-10)
    X, info = hpw.solve_complex(torch.from_numpy(A).cuda(), alpha_rule="user", alpha=alpha,
                                variant=variant, tol=1e-10)
    torch.cuda.synchronize()
    Xh = X.cpu().numpy()
    say(f"  {info['status']} iters {info['iters']} (oracle {ref.iters})")
    assert info["status"] == ref.status == "ok"
    assert info["iters"] == ref.iters
    assert rel(Xh, ref.X) <= 1e-10
    assert rel(Xh, np.linalg.pinv(A)) <= 1e-10
    for r in O.penrose_residuals(A, Xh):
        assert r < 1e-10


def test_complex_default_alpha_and_rejected_rules():
    hpw = need_gpu()
    A = complex_input(90, 60, 60, seed=3)
    X, info = hpw.solve_complex(torch.from_numpy(A).cuda(), tol=1e-10)
    torch.cuda.synchronize()
    assert info["status"] == "ok"
    assert rel(X.cpu().numpy(), np.linalg.pinv(A)) <= 1e-10
    Sq = complex_input(40, 40, 40, seed=4)
    for kw in (dict(kind="drazin", l=1), dict(alpha_rule="diag")):
        with pytest.raises(hpw.HyperpowerError) as e:
            hpw.solve_complex(torch.from_numpy(Sq).cuda(), **kw)
        assert e.value.code == hpw.HP_EUNSUPPORTED
