"""The seeded generators hit the spectra, ranks and indices they promise."""

import numpy as np

from paper_1604_07893_amd import inputs


def test_uniform_is_seeded_and_bounded():
    a = inputs.uniform(200, 100, seed=1001)
    b = inputs.uniform(200, 100, seed=1001)
    assert a.shape == (200, 100) and np.array_equal(a, b)
    assert a.min() >= -1 and a.max() <= 1
    assert np.linalg.matrix_rank(a) == 100


def test_lowrank_svd_spectrum_and_rank():
    d = inputs.lowrank_svd(256, 128, 96, smin=1e-4, seed=3)
    s = np.linalg.svd(d.A, compute_uv=False)
    assert abs(s[0] - 1.0) < 1e-12
    assert np.allclose(s[:96], d.s, rtol=1e-9, atol=1e-14)
    assert s[96] < 1e-14
    assert np.allclose(d.U.T @ d.U, np.eye(96), atol=1e-13)
    assert np.allclose(d.V.T @ d.V, np.eye(96), atol=1e-13)


def test_square_svd_condition():
    d = inputs.square_svd(128, smin=1e-3, seed=4)
    s = np.linalg.svd(d.A, compute_uv=False)
    assert abs(s[0] - 1) < 1e-12 and abs(s[-1] - 1e-3) < 1e-12
    assert np.all(np.diff(d.s) <= 0)


def test_drazin_jordan_index_and_spectrum():
    d = inputs.drazin_jordan(n=64, nb=52, cond_p=10.0, seed=5)
    assert d.index == 3
    assert np.allclose(d.P @ d.Pinv, np.eye(64), atol=1e-12)
    assert np.linalg.cond(d.P) < 10.0 + 1e-6
    ranks = [np.linalg.matrix_rank(np.linalg.matrix_power(d.A, k), tol=1e-8) for k in range(5)]
    # 12 nilpotent rows in blocks of 3: ranks drop by 4 per power until index 3
    assert ranks == [64, 60, 56, 52, 52]
    assert d.lam.min() >= 0.5 and d.lam.max() <= 2.0


def test_request_stream_shapes():
    reqs = inputs.request_stream(200, qps=100.0, seed=6)
    assert all(64 <= r.A.shape[0] <= 2048 for r in reqs)
    assert all(r.A.shape[0] % 4 == 0 for r in reqs)
    assert all(r.A.shape[0] // r.A.shape[1] in (1, 2, 4) for r in reqs)
    t = [r.arrival_s for r in reqs]
    assert all(b > a for a, b in zip(t, t[1:]))
    frac = np.mean([r.rank_deficient for r in reqs])
    assert 0.02 < frac < 0.2
    r = next(r for r in reqs if r.rank_deficient)
    assert np.linalg.matrix_rank(r.A) == max(1, min(r.A.shape) // 2)


def test_hilbert():
    h = inputs.hilbert(5, 3)
    assert h[0, 0] == 1 and abs(h[4, 2] - 1 / 7) < 1e-16
