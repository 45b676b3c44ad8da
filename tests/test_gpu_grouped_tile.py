"""The tile of the grouped launch of batched and served solves: each of the
three tile configurations (forced through hp_tune_import), and the one
hp_autotune picks, keep a batched result equal to the same problem solved
alone (bitwise), served results equal to batched ones, and the oracle parity
of the batched form (Section 4's Moore-Penrose iteration, stabilised)."""

import numpy as np
import pytest
import torch

import oracle as O
from gpu_common import need_gpu, rel, say, to_dev
from paper_1604_07893_amd import inputs

pytestmark = pytest.mark.gpu

KW = dict(variant="stabilised", tol=1e-12, precision="fp32_fp64")


def problems(seed):
    rng = np.random.default_rng(seed)
    shapes = [(64, 64, False), (130, 65, False), (65, 130, False), (257, 129, False),
              (300, 75, False), (96, 96, True), (200, 100, True), (33, 17, False)]
    return [inputs.request_matrix(rng, m, n, d) for m, n, d in shapes]


@pytest.fixture
def hpw():
    h = need_gpu()
    yield h
    # later tests see the default tile again
    h.import_tuning([(h.GEMM_DTYPES["grouped_f64"], 0, 0, 0, 0),
                     (h.GEMM_DTYPES["grouped_f32"], 0, 0, 0, 0)])


def force(hpw, cfg):
    hpw.import_tuning([(hpw.GEMM_DTYPES["grouped_f64"], 0, 0, 0, cfg),
                       (hpw.GEMM_DTYPES["grouped_f32"], 0, 0, 0, cfg)])


def check_group(hpw, As, label):
    dev = [to_dev(a) for a in As]
    Xs, infos = hpw.solve_batched(dev, **KW)
    torch.cuda.synchronize()
    for A, X, info in zip(As, Xs, infos):
        ref = O.solve(A, kind="mp", variant="stabilised", tol=1e-12)
        err = rel(X.cpu().numpy(), ref.X)
        say(f"  {label} {A.shape} {info['status']} stages {info['iters_stage']} err {err:.2e}")
        assert info["status"] in ("ok", "stagnated")
        assert err <= 1e-10
    for i in (0, 3, 7):
        Xa, _ = hpw.solve_batched([dev[i]], **KW)
        assert torch.equal(Xa[0], Xs[i]), (label, i)
    # the server runs the same grouped loop: same results, bitwise
    srv = hpw.Server(hbm_budget=1 << 28, max_slots=16, **KW)
    tick = [srv.submit(a) for a in dev]
    got = {}
    for _ in range(500):
        srv.step()
        for j, t in enumerate(tick):
            if j not in got:
                r = srv.poll(t)
                if r is not None:
                    got[j] = r[0]
        if len(got) == len(tick):
            break
    srv.close()
    assert len(got) == len(tick)
    for j in range(len(tick)):
        assert torch.equal(got[j], Xs[j]), (label, "served", j)


@pytest.mark.parametrize("cfg", [0, 1, 2])
def test_forced_grouped_tile(hpw, cfg):
    say(f"grouped tile {hpw.GROUPED_TILES[cfg]}")
    force(hpw, cfg)
    check_group(hpw, problems(60 + cfg), f"cfg{cfg}")


def test_autotuned_grouped_tile(hpw):
    picks = {}
    for name in ("grouped_f64", "grouped_f32"):
        (M, N, K, t, ms), = hpw.autotune([(256, 256, 512)], dtype=name, reps=3)
        say(f"autotune {name} 256x256x512: tile {t} ({hpw.GROUPED_TILES[t]}) {ms * 1e3:.1f} us")
        assert t in hpw.GROUPED_TILES and ms > 0
        picks[name] = t
        rows = hpw.tuning_table()
        assert (hpw.GEMM_DTYPES[name], 256, 256, 512, t) in rows
    check_group(hpw, problems(70), f"tuned{picks['grouped_f64']}/{picks['grouped_f32']}")


def test_tune_import_rejects_bad_grouped_rows(hpw):
    for row in ((hpw.GEMM_DTYPES["grouped_f64"], 0, 0, 0, 3),
                (hpw.GEMM_DTYPES["grouped_f32"], 0, 0, 0, -1), (8, 1, 1, 1, 0)):
        with pytest.raises(hpw.HyperpowerError):
            hpw.import_tuning([row])
