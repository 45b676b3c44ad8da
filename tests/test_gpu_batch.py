"""Batched (grouped launches) and served (continuous batching) forms against
the oracle, plus the alone-vs-in-mix identity of each result."""

import numpy as np
import pytest
import torch

import oracle as O
from gpu_common import need_gpu, rel, say, to_dev
from paper_1604_07893_amd import inputs

pytestmark = pytest.mark.gpu


def mixed_problems(seed=40):
    rng = np.random.default_rng(seed)
    shapes = [(64, 64, False), (130, 65, False), (65, 130, False), (257, 129, False),
              (300, 75, False), (96, 96, True), (200, 100, True), (128, 128, False)]
    return [inputs.request_matrix(rng, m, n, d) for m, n, d in shapes]


@pytest.mark.parametrize("precision", ["fp64", "fp32_fp64"])
def test_batched_matches_oracle(precision):
    hpw = need_gpu()
    say(f"batched {precision}")
    As = mixed_problems()
    Xs, infos = hpw.solve_batched([to_dev(a) for a in As], variant="stabilised", tol=1e-12,
                                  precision=precision)
    torch.cuda.synchronize()
    for A, X, info in zip(As, Xs, infos):
        ref = O.solve(A, kind="mp", variant="stabilised", tol=1e-12)
        ref_p = np.linalg.pinv(A, rcond=1e-10)
        err = rel(X.cpu().numpy(), ref.X)
        say(f"  {A.shape} {info['status']} iters {info['iters']} stages {info['iters_stage']} "
            f"err {err:.2e} vs pinv {rel(X.cpu().numpy(), ref_p):.2e}")
        assert info["status"] in ("ok", "stagnated")
        assert err <= 1e-10
        assert rel(X.cpu().numpy(), ref_p) <= 1e-9


def test_batched_alone_equals_in_mix_bitwise():
    hpw = need_gpu()
    As = mixed_problems(41)
    dev = [to_dev(a) for a in As]
    Xs, _ = hpw.solve_batched(dev, variant="stabilised", tol=1e-12, precision="fp32_fp64")
    for i in (0, 3, 6):
        Xa, _ = hpw.solve_batched([dev[i]], variant="stabilised", tol=1e-12, precision="fp32_fp64")
        assert torch.equal(Xa[0], Xs[i]), i


def test_server_continuous_batching_and_budget():
    """Requests submitted while others run are admitted as memory frees up;
    every result equals the same request served alone (bitwise) and matches
    the oracle."""
    hpw = need_gpu()
    rng = np.random.default_rng(42)
    shapes = [(256, 128), (512, 512), (64, 64), (384, 96), (128, 256), (200, 200), (96, 48)]
    As = [rng.standard_normal(s) for s in shapes]
    kw = dict(variant="stabilised", tol=1e-12, precision="fp32_fp64")
    need = [hpw.workspace_bytes(hpw.make_params(**kw), *s) for s in shapes]
    budget = int(1.2 * max(need)) + (1 << 20)  # below the sum: forces waiting and reuse
    assert budget < sum(need)
    srv = hpw.Server(hbm_budget=budget, max_slots=4, **kw)
    tickets = []
    done = {}
    max_active, saw_waiting = 0, False
    for i, A in enumerate(As):
        tickets.append(srv.submit(to_dev(A)))
        if i % 2 == 1:  # interleave arrivals with steps
            a, w = srv.step()
            max_active, saw_waiting = max(max_active, a), saw_waiting or w > 0
    steps = 0
    while len(done) < len(As) and steps < 500:
        a, w = srv.step()
        max_active, saw_waiting = max(max_active, a), saw_waiting or w > 0
        steps += 1
        for i, t in enumerate(tickets):
            if i not in done:
                r = srv.poll(t)
                if r is not None:
                    done[i] = r
    srv.close()
    assert len(done) == len(As)
    assert 1 <= max_active <= 4 and saw_waiting
    for i, A in enumerate(As):
        X, info = done[i]
        assert info["status"] in ("ok", "stagnated")
        ref = O.solve(A, kind="mp", variant="stabilised", tol=1e-12)
        assert rel(X.cpu().numpy(), ref.X) <= 1e-10
        assert info["queue_ms"] >= 0 and info["run_ms"] > 0
        alone = hpw.Server(hbm_budget=budget, max_slots=4, **kw)
        t = alone.submit(to_dev(A))
        r = None
        while r is None:
            alone.step()
            r = alone.poll(t)
        alone.close()
        assert torch.equal(r[0], X), i


def test_server_rejects_request_over_budget():
    hpw = need_gpu()
    srv = hpw.Server(hbm_budget=1 << 20, max_slots=2, precision="fp64")
    with pytest.raises(hpw.HyperpowerError) as e:
        srv.submit(torch.zeros((1024, 1024), dtype=torch.float64, device="cuda:0"))
    assert e.value.code == hpw.HP_EBUDGET
    srv.close()


def test_single_fp32_fp64_rectangular_uses_projection():
    """FP32 loops then FP64 loops on a rectangular input reach FP64 accuracy
    (the projection onto the Penrose conditions removes the FP32 error left in
    the blocks the iteration does not correct)."""
    hpw = need_gpu()
    rng = np.random.default_rng(43)
    for (m, n, d) in [(512, 256, False), (300, 150, True), (150, 300, False)]:
        A = inputs.request_matrix(rng, m, n, d)
        ref = np.linalg.pinv(A, rcond=1e-10)
        X, info = hpw.solve(to_dev(A), variant="stabilised", precision="fp32_fp64", tol=1e-12)
        err = rel(X.cpu().numpy(), ref)
        say(f"  {m}x{n} deficient={d} stages {info['iters_stage']} err {err:.2e}")
        assert err <= 1e-10


def test_graph_replay_matches_eager_launches():
    """Every loop of a batch replays the captured graph; the results equal
    those of launching the same kernels one by one, bitwise, for every
    problem (so each of the ~10 replays reproduced the eager loop)."""
    hpw = need_gpu()
    As = [to_dev(a) for a in mixed_problems(44)]
    kw = dict(variant="stabilised", tol=1e-12, precision="fp32_fp64")
    Xg, ig = hpw.solve_batched(As, graph=True, **kw)
    Xe, ie = hpw.solve_batched(As, graph=False, **kw)
    for a, b, i1, i2 in zip(Xg, Xe, ig, ie):
        assert i1["iters"] == i2["iters"] and i1["iters"] >= 3
        assert torch.equal(a, b)


def test_ill_conditioned_square_requests_stay_accurate():
    """Square N(0,1) requests of the served stream (kappa ~ 1e3) whose change
    rises and falls around 1 under the FP32 loops: a stage exit during that
    transient, followed by the Penrose projection, used to return a wrong
    result flagged "stagnated". Single solves and a batch, FP32 then FP64."""
    reqs = inputs.request_stream(1100, qps=1.0, seed=1005)
    picks = [75, 344, 1068]
    mats = [reqs[i].A for i in picks]
    for A in mats:
        assert A.shape[0] == A.shape[1] and not np.any(np.isnan(A))
    hpw = need_gpu()
    kw = dict(variant="stabilised", tol=1e-10, precision="fp32_fp64")
    for A in mats:
        X, info = hpw.solve(to_dev(A), **kw)
        torch.cuda.synchronize()
        P = np.linalg.pinv(A)
        say(f"  single {A.shape} {info['status']} stages {info['iters_stage']}")
        assert info["status"] == "ok"
        assert rel(X.cpu().numpy(), P) <= 1e-10
    Xs, infos = hpw.solve_batched([to_dev(A) for A in mats], **kw)
    torch.cuda.synchronize()
    for A, X, info in zip(mats, Xs, infos):
        assert info["status"] == "ok"
        assert rel(X.cpu().numpy(), np.linalg.pinv(A)) <= 1e-10


@pytest.mark.parametrize("retry", [True, False])
def test_server_retries_a_failed_request_in_fp64(retry):
    """A request with entries near 1e45: beyond FP32's range (the FP32 loop is
    non-finite) and with X0 = alpha A^T near 1e-49, below FP32's smallest
    subnormal, so the FP64 stage starts from X = 0 and ends non-finite too.
    The server runs it once more in FP64 only (default), which reaches the
    pseudo-inverse; with HP_FLAG_NO_RETRY the failure is reported. Its
    neighbour is unaffected."""
    hpw = need_gpu()
    rng = np.random.default_rng(4)
    A_ok = rng.standard_normal((96, 64))
    A_big = rng.standard_normal((80, 80)) * 1e45
    srv = hpw.Server(hbm_budget=1 << 28, max_slots=4, precision="fp32_fp64", tol=1e-10,
                     variant="stabilised", retry=retry)
    t1, t2 = srv.submit(to_dev(A_ok)), srv.submit(to_dev(A_big))
    results = {}
    for _ in range(400):
        srv.step()
        for t in (t1, t2):
            if t not in results:
                r = srv.poll(t)
                if r is not None:
                    results[t] = r
        if len(results) == 2:
            break
    srv.close()
    assert len(results) == 2
    (X1, i1), (X2, i2) = results[t1], results[t2]
    say(f"  retry={retry}: {i1['status']} {i2['status']} stages {i2['iters_stage']}")
    assert i1["status"] == "ok"
    assert rel(X1.cpu().numpy(), np.linalg.pinv(A_ok)) <= 1e-10
    if retry:
        assert i2["status"] == "ok" and list(i2["iters_stage"][:2]) == [0, 0]
        assert rel(X2.cpu().numpy(), np.linalg.pinv(A_big)) <= 1e-10
    else:
        assert i2["status"] != "ok"
