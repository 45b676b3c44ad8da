"""hp_params.device_stop: the stop / switch / guard decisions taken on the
device (the rules of Section 4's stopping test, the switch recipe of Section 7,
the guards of Section 6) with the loops enqueued in chunks. The decisions and
iterates must be those of the host-driven loop, bit for bit: same status, loop
count, switch loop, change history and X."""

import numpy as np
import pytest
import torch

import oracle as O
from gpu_common import need_gpu, rel, say, to_dev
from paper_1604_07893_amd import inputs

pytestmark = pytest.mark.gpu


def both(A, **kw):
    hpw = need_gpu()
    Ad = to_dev(A) if isinstance(A, np.ndarray) else A
    X0, i0 = hpw.solve(Ad, device_stop=False, **kw)
    X1, i1 = hpw.solve(Ad, device_stop=True, **kw)
    torch.cuda.synchronize()
    return X0, i0, X1, i1


def same(X0, i0, X1, i1):
    assert i1["status"] == i0["status"]
    assert i1["iters"] == i0["iters"]
    assert i1["switch_iter"] == i0["switch_iter"]
    assert i1["d_hist"] == i0["d_hist"]
    assert i1["gemms"] == i0["gemms"]
    assert abs(i1["gflop"] - i0["gflop"]) <= 1e-9 * max(i0["gflop"], 1.0)
    assert torch.equal(X1, X0)


def test_200x100_moore_penrose_matches_host_loop_and_oracle():
    A = inputs.uniform(200, 100, seed=1001)
    X0, i0, X1, i1 = both(A, tol=1e-12)
    say(f"200x100: {i1['status']} iters {i1['iters']} (host {i0['iters']})")
    same(X0, i0, X1, i1)
    ref = O.solve(A, kind="mp", tol=1e-12)
    assert i1["iters"] == ref.iters and rel(X1.cpu().numpy(), ref.X) <= 1e-10


@pytest.mark.parametrize("side", ["right", "left"])
def test_stabilised_switch_on_rank_deficient_input(side):
    d = inputs.lowrank_svd(320, 160, 120, smin=1e-3, seed=12)
    X0, i0, X1, i1 = both(d.A, alpha_rule="user", alpha=1.0, variant="stabilised", tol=1e-10,
                          side=side)
    say(f"rank-deficient {side}: {i1['status']} iters {i1['iters']} switch {i1['switch_iter']}")
    assert i1["switch_iter"] > 0
    same(X0, i0, X1, i1)


@pytest.mark.parametrize("variant", ["plain", "stabilised"])
@pytest.mark.parametrize("n,nb", [(256, 224), (2048, 1792)])
def test_drazin_plain_and_stabilised(variant, n, nb):
    dz = inputs.drazin_jordan(n=n, nb=nb, cond_p=10.0, seed=1004)
    X0, i0, X1, i1 = both(dz.A, kind="drazin", l=3, variant=variant, tol=1e-10)
    say(f"drazin {n} {variant}: {i1['status']} iters {i1['iters']}")
    same(X0, i0, X1, i1)


def test_large_products_on_the_load_to_lds_tile():
    """3072^2 (576 tiles of 128^2): the products run on the load-to-LDS FP64
    tile, whose launches are gated like the others. Decisions and X bitwise
    those of the host loop."""
    d = inputs.square_svd(3072, smin=1e-3, seed=3073)
    X0, i0, X1, i1 = both(d.A, alpha_rule="user", alpha=1.0, tol=1e-10)
    say(f"3072^2: {i1['status']} iters {i1['iters']}")
    same(X0, i0, X1, i1)
    closed = (d.V / d.s) @ d.U.T
    assert i1["status"] == "ok" and rel(X1.cpu().numpy(), closed) <= 1e-10


def test_guards_and_loop_cap():
    A = inputs.uniform(90, 60, seed=4)
    s1 = np.linalg.svd(A, compute_uv=False)[0]
    # alpha sigma_1^2 = 4: diverges; the best iterate before the blow-up
    X0, i0, X1, i1 = both(A, alpha_rule="user", alpha=4.0 / s1**2, tol=1e-12)
    assert i1["status"] == "diverged"
    same(X0, i0, X1, i1)
    # the loop cap
    X0, i0, X1, i1 = both(A, tol=1e-12, max_iter=3)
    assert i1["status"] == "maxiter" and i1["iters"] == 3
    same(X0, i0, X1, i1)
    # plain loops on rank-deficient input stop at the stagnation guard
    d = inputs.lowrank_svd(120, 60, 40, smin=1e-3, seed=6)
    X0, i0, X1, i1 = both(d.A, alpha_rule="user", alpha=1.0, tol=1e-13)
    assert i1["status"] == "stagnated"
    same(X0, i0, X1, i1)


@pytest.mark.parametrize("stop,tol", [("paper_4_1", 1e-6), ("abs_inf", 1e-9)])
def test_other_stopping_rules(stop, tol):
    A = inputs.uniform(120, 80, seed=3)
    X0, i0, X1, i1 = both(A, stop=stop, tol=tol, inf_norm=True)
    assert i1["status"] == "ok"
    same(X0, i0, X1, i1)
    assert i1["dinf_hist"] == i0["dinf_hist"]


def test_comparison_schemes():
    A = inputs.square_svd(128, smin=1e-2, seed=8).A
    for method in ("sm", "cm", "fm", "hm"):
        X0, i0, X1, i1 = both(A, method=method, alpha_rule="user", alpha=1.0, tol=1e-11)
        assert i1["status"] == "ok", method
        same(X0, i0, X1, i1)


def test_launched_loop_by_loop_and_without_allocation():
    """The same decisions without the captured graph (HP_FLAG_NO_GRAPH), and
    through hp_solve_noalloc (which never captures)."""
    hpw = need_gpu()
    A = inputs.uniform(200, 100, seed=1001)
    X0, i0, X1, i1 = both(A, tol=1e-12, graph=False)
    same(X0, i0, X1, i1)
    Ad = to_dev(A)
    Xn = torch.empty_like(X0)
    i2 = hpw.solve_noalloc(Ad, Xn, tol=1e-12, device_stop=True)
    torch.cuda.synchronize()
    same(X0, i0, Xn, i2)


def test_cached_graph_follows_a_new_workspace_and_tolerance():
    """The graph of two loops is cached per workspace: a second solve on the
    same workspace with another tolerance, and one on a new workspace, both
    reproduce the host-driven loop."""
    hpw = need_gpu()
    A = to_dev(inputs.uniform(150, 90, seed=21))
    nbytes = hpw.workspace_bytes(hpw.make_params(), 150, 90)
    for ws in (torch.empty(nbytes, dtype=torch.uint8, device=A.device),
               torch.empty(nbytes + 4096, dtype=torch.uint8, device=A.device)):
        for tol in (1e-6, 1e-12):
            X0, i0 = hpw.solve(A, workspace=ws, tol=tol)
            X1, i1 = hpw.solve(A, workspace=ws, tol=tol, device_stop=True)
            torch.cuda.synchronize()
            same(X0, i0, X1, i1)


def test_latency_200x100():
    """Reported, not asserted: microseconds per inverse with the host reading
    the stopping sums after every loop and with the decisions on the device."""
    hpw = need_gpu()
    A = to_dev(inputs.uniform(200, 100, seed=1001))
    out = torch.empty((100, 200), dtype=torch.float64, device=A.device)
    ws = torch.empty(hpw.workspace_bytes(hpw.make_params(), 200, 100), dtype=torch.uint8,
                     device=A.device)
    import time
    for flag, graph in ((False, True), (True, True), (True, False)):
        for _ in range(5):
            hpw.solve(A, out=out, workspace=ws, tol=1e-12, device_stop=flag, graph=graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(50):
            hpw.solve(A, out=out, workspace=ws, tol=1e-12, device_stop=flag, graph=graph)
        torch.cuda.synchronize()
        say(f"200x100 device_stop={flag} graph={graph}: "
            f"{(time.perf_counter() - t0) / 50 * 1e6:.0f} us")
