"""The residual-bound stopping rule (HP_STOP_REL_FRO_BOUND) on the GPU against
the same rule in the CPU oracle: before a plain final-stage loop that follows a
change d with d^p < tol, ||R||_F / (1 - ||R||_F) < tol bounds that loop's
change below tol, so X_{k+1} is returned without running it."""

import numpy as np
import pytest
import torch

import oracle as O
from gpu_common import need_gpu, rel, say, to_dev
from paper_1604_07893_amd import inputs

pytestmark = pytest.mark.gpu

PRODUCTS = {"sm": 2, "cm": 3, "fm": 5, "hm": 9, "pm": 7}


def run(A, **kw):
    hpw = need_gpu()
    X, info = hpw.solve(to_dev(A), **kw)
    torch.cuda.synchronize()
    return X.cpu().numpy(), info


@pytest.mark.parametrize("method,smin,seed", [("pm", 1e-2, 21), ("sm", 1e-2, 21), ("cm", 1e-2, 21),
                                               ("fm", 1e-2, 21), ("hm", 1e-2, 21), ("pm", 1e-1, 30)])
def test_bound_rule_matches_oracle_square(method, smin, seed):
    """(smin 1e-1, seed 30: the check before the last loop does not settle, and
    that loop runs SM, X + X R on the residual already formed.)"""
    say(f"bound rule {method} smin {smin} seed {seed}")
    d = inputs.square_svd(256, smin=smin, seed=seed)
    closed = (d.V / d.s) @ d.U.T
    ref = O.solve(d.A, kind="mp", method=method, stop="rel_fro_bound", tol=1e-10)
    plain = O.solve(d.A, kind="mp", method=method, stop="rel_fro", tol=1e-10)
    X, info = run(d.A, method=method, stop="rel_fro_bound", tol=1e-10)
    assert info["status"] == ref.status == "ok"
    assert info["iters"] == ref.iters
    skipped = ref.iters < plain.iters
    # one residual product per bound check (reused by the loop if it runs)
    checks = len(ref.bound_hist)
    # each loop runs the scheme the oracle ran (a check that does not settle
    # hands its residual product to the loop after it)
    assert info["gemms"] == sum(PRODUCTS[m] for m in ref.method_hist) + (1 if skipped else 0)
    assert checks >= (1 if skipped else 0)
    assert rel(X, ref.X) <= 1e-10
    assert rel(X, closed) <= 1e-12
    if skipped:
        assert info["stop_last"] < 1e-10


def test_bound_rule_is_inert_on_rank_deficient_input():
    """R = I - XA tends to a projector of norm >= 1: the rule is the relative
    change there."""
    lr = inputs.lowrank_svd(240, 120, 80, smin=1e-3, seed=6)
    ref = O.solve(lr.A, kind="mp", variant="stabilised", stop="rel_fro", tol=1e-10)
    X, info = run(lr.A, variant="stabilised", stop="rel_fro_bound", tol=1e-10)
    assert info["status"] == "ok" and info["iters"] == ref.iters
    assert rel(X, ref.X) <= 1e-9


@pytest.mark.parametrize("precision", ["mixed", "fp32_fp64"])
def test_bound_rule_saves_the_confirming_fp64_loop(precision):
    say(f"bound rule {precision}")
    d = inputs.square_svd(384, smin=1e-3, seed=31)
    closed = (d.V / d.s) @ d.U.T
    kw = dict(precision=precision, alpha_rule="user", alpha=1.0, tol=1e-10)
    X0, info0 = run(d.A, stop="rel_fro", **kw)
    X1, info1 = run(d.A, stop="rel_fro_bound", **kw)
    say(f"  stages {info0['iters_stage']} -> {info1['iters_stage']}")
    assert info0["status"] == info1["status"] == "ok"
    assert info1["iters_stage"][:2] == info0["iters_stage"][:2]
    assert info1["iters_stage"][2] == info0["iters_stage"][2] - 1
    assert rel(X1, closed) <= 1e-11
    assert rel(X0, closed) <= 1e-11


def test_bound_rule_fp32_final_stage():
    d = inputs.square_svd(200, smin=1e-1, seed=41)
    closed = (d.V / d.s) @ d.U.T
    X, info = run(d.A, precision="fp32", stop="rel_fro_bound", alpha_rule="user", alpha=1.0,
                  tol=1e-5)
    assert info["status"] == "ok"
    assert rel(X, closed) <= 1e-5


@pytest.mark.parametrize("r1", [0.3, 0.6, 0.75])
def test_bound_rule_scheme_choice_matches_oracle(r1):
    """The loop after a residual check that does not settle runs SM, CM or FM
    on the residual already formed (X + XR, X(I + R + R^2), FM's products):
    same schemes, product count and result as the oracle's rule."""
    say(f"bound scheme r1={r1}")
    d = inputs.square_svd(128, smin=1e-3, seed=51)
    r = np.zeros(128)
    r[np.argmax(d.s)] = r1
    X0 = (d.V * ((1 - r) / d.s)) @ d.U.T
    ref = O.solve(d.A, X0=X0, stop="rel_fro_bound", tol=1e-10)
    X, info = run(d.A, X0=to_dev(X0), stop="rel_fro_bound", tol=1e-10)
    say(f"  oracle schemes {ref.method_hist} gemms {info['gemms']}")
    assert info["status"] == ref.status == "ok"
    assert info["iters"] == ref.iters
    settled_by_check = len(ref.bound_hist) > len(ref.method_hist) - 1
    assert info["gemms"] == sum(PRODUCTS[m] for m in ref.method_hist) + (1 if settled_by_check else 0)
    closed = (d.V / d.s) @ d.U.T
    assert rel(X, ref.X) <= 1e-10 and rel(X, closed) <= 1e-12
